// Internal declarations shared by the host side and the kernels of libpbsplit.
//
// Device layout of one generation of fluence (element type T = float|double):
//   psi[g][l][pb][a][pt]      g = energy group, l = DG coefficient (0: psi^1, 1: psi^2),
//                             a = i*m + j interior angular node (m = nth-1),
//                             lateral cell pq = p*ny + q split as pb = pq / PT, pt = pq % PT.
// A "line" is one (pb, a, pt) triple: line = (pb*NA + a)*PT + pt; the (g, l) slab of a
// generation is contiguous, so element (g, l, line) sits at (g*2 + l)*NLINE + line.
// Source and scan buffers use [state][g][line].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PBS_PT 32            // lateral tile: 32 consecutive cells = 128 B of FP32
#define PBS_MAX_NSEG 4       // transport sweep supports ny <= 64 * PBS_MAX_NSEG
#define PBS_KPB_ALIGN 64     // source-node padding of the split-BF16 transfer matrix (the K stage)
#ifndef PBS_EPASS_LPT
#define PBS_EPASS_LPT 4      // angular lines per thread of the split-scan energy pass (4 or 8)
#endif

namespace pbs {

enum { MODE_CLOSE = 1, MODE_OPEN = 2, MODE_PAIR = 3 };

template <typename T>
struct EParams {
    T *psi;                 // one generation
    const T *Q;             // [2][G][NLINE] source without the density factor, Q^n + Q* of the closing (0)
                            // and opening (1) half-step, or null
    const unsigned short *Qb = nullptr;   // the same source in BF16, [2][G][NPB][NAq / 4][PT][4] with
                                          // NAq = NA rounded up to 4 (a = 4 a4 + e), which then replaces Q
    T *W;                   // [2][G][NLINE] energy-scanned psi^1 of this generation, summed over the two
                            // states of each half-step (0: close, 1: open), or null
    unsigned short *Wh, *Wl;   // split-BF16 form of W (hi, lo): [2][G][NPB][NOCT][PT][8], a' = 8*oct + e;
                               // Wl null: hi only
    int NOCT;                  // ceil(NA / 8)
    const T *rho_c;         // densities of the closing half-step layer [NPpad] (MODE_CLOSE bit)
    const T *rho_o;         // densities of the opening half-step layer [NPpad] (MODE_OPEN bit)
    double *dep_c;          // [NLINE] deposited energy of the closing half-step (MeV)
    double *dep_o;          // [NLINE] deposited energy of the opening half-step
    const T *Sm, *Sp, *kap; // S_{g-1/2}/dE_g, S_{g+1/2}/dE_g, kappa_g
    const T *wc, *wdec, *invdE;   // energy re-emission scan: weight, decay to g-1, 1/dE_g
    const double *dA, *dB, *dInj; // deposit functional weights (per group)
    double dBot;            // S_{1/2} E_{1/2}: energy carried through the bottom face
    double scale;           // dth^2 dx dy
    T h;                    // length of each CN half-step
    int G;
    long NLINE, NAPT;       // lines per (g,l) slab; NA*PT
    // surrogate features of this generation (all null unless recorded): per line, the energy that
    // the closing / opening half-step injects into the next generation (MeV, FP64) and the energy
    // and number moments of psi^1 after the opening half-step
    double *inj_c = nullptr, *inj_o = nullptr, *mom_e = nullptr, *mom_n = nullptr;
    const double *wmom = nullptr;   // [3G] moment weights: E_g dE_g and dE_g^2/6 (energy), dE_g (number) at G + g
    // nuclear bands (NB > 1): the scan is a sum of per-band scans with the source group's decay,
    // U^b_g = [band_g = b] wc_g psi1_g + wdecb[b*G + g] U^b_{g+1}
    int NB = 1;
    const int *band = nullptr;
    const T *wdecb = nullptr;
    // straggling (blk non-null): rho-free 2x2 blocks [G][12] (Lo, Di, Up), per-cell elimination factors of
    // the closing / opening half-step sfac[g][8][NPpad] (Dinv row-major, then F = a Up Dinv_{g+1}), and the
    // deposit weights of psi1, psi2 of the whole operator
    const T *blk = nullptr;
    T *sfac_c = nullptr, *sfac_o = nullptr;
    const double *dA2 = nullptr, *dB2 = nullptr;
    long NPpad = 0;
};

template <typename T>
struct TParams {
    T *psi;                 // base of the planes (generation 0)
    const T *theta;         // [m] angular coordinates of the interior nodes
    T h_half_over_dx, h_half_over_dy;   // h/(2 dx), h/(2 dy)
    int nx, ny, m, NA;
    long NLINE;
    long nplanes;           // ngen*G*2*NA
};

template <typename T>
struct AParams {
    T *psi;
    const T *rho;           // [NPpad] densities of the layer
    const T *sig;           // [G] group-mean scattering power
    const T *S;             // [(N-1)*(N-1)] sin(pi M n / N)
    const T *lam;           // [N-1] (2cos(pi M/N) - 2)/dth^2
    T h;                    // CN step length
    int G, NA, NPB;
    long NLINE;
};

template <typename T>
struct QParams {
    const T *P2T;           // [NA][NA]: P2T[a][a'] = probability a' -> a
    const T *W;             // [2][G][NLINE]
    T *Q;                   // [2][G][NLINE]
    unsigned short *Qb = nullptr;   // non-null: write the source in BF16 there instead (EParams::Qb layout)
    const T *P2p;           // [Kp][Mp] zero-padded P2 (k = source node, row = destination), MFMA path
    int Kp, Mp;
    const unsigned short *Bh, *Bl;   // split-BF16 W (see EParams), split-BF16 path
    int NOCT;
    int NA, NPB, G;
    int s0, ns;             // half-step sums s0 .. s0+ns-1
    long NLINE;
    const int *band = nullptr;   // nuclear band of every destination group (null: one band); the transfer
                                 // matrices of the bands follow each other (P2T, P2p, split tables)
};

// One beam of a batch (device copy of its descriptor).  Beams of one batch share the lateral and
// angular grid and the number of generations; groups, depth steps and step length differ.
struct BeamDev {
    float *psi;               // generation 0 of the fluence; generations follow
    float *Q;                 // [2][G][NLINE]
    unsigned short *Wh, *Wl;  // split-BF16 energy scans, [2][G][NPB][NOCT][PT][8]
    const float *rho;         // [nz][NPB*PT]
    double *dep;              // [2][ngen][NLINE]
    double *edep;             // [nz][NP]
    const float *tabf;        // Sm, Sp, kappa, wc, wdec, 1/dE, sigma_tr: 7 arrays of G
    const double *tabd;       // deposit weights dA, dB, dInj: 3 arrays of G
    double dBot;
    float dz;
    float thx, thy;           // transport factors (dz/4)/dx, (dz/4)/dy, rounded once from FP64 as in the
                              // single-beam path so a batched beam is bitwise the single-beam run
    int G, nz;
};

struct BatchShape {
    const float *theta, *lam, *S;          // angular tables
    const float *K;                        // MFMA operand table of the angular pass (nth 16 or 32)
    const unsigned short *Ahi, *Alo;       // split-BF16 P2, [Mp][Kpb]
    int Kpb, Mp;
    int nprod;                             // 3: scanned fluence as hi + lo; 2: hi only (no lo array);
                                           // 1: hi only, with the compensated single-BF16 matrix as Ahi
    int nx, ny, nth, m, NA, NPB, NOCT, ngen;
    long NLINE;
    float dx, dy;
    double scale;                          // dth^2 dx dy
};

// bitwise-neutral launch variants picked by the batch autotuner
struct BatchTuning {
    int gemm_kind = 0;        // split-BF16 product kernel (QGEMM_*)
    int tpass_wpb = 4;        // transport: planes (waves) per block, 1, 2 or 4
    int apass_pc = 32;        // angular pass: lateral cells per block, 8, 16 or 32
    int max_nz = 0;           // longest beam of the wave (set by the batch planner)
};

// Side stream of a batch march: each generation's T A T runs there after its energy pass (events per
// generation; pend marks a T A T that the main stream has not waited for yet).
struct BatchSide {
    hipStream_t side;
    hipEvent_t *ev_e, *ev_tat;
    char *pend;
};

// One fused depth step s of a wave.  Without sd every sub-step runs on st in order.
hipError_t launch_batch_step(const BeamDev *beams, int nbeam, const BatchShape &Sh, int s, int maxG,
                             const BatchTuning &tu, hipStream_t st, const BatchSide *sd = nullptr);

// launchers (explicitly instantiated for float and double); return hipGetLastError()
template <typename T> hipError_t launch_epass(const EParams<T> &P, int mode, hipStream_t st);
// energy pass with straggling (P.blk set): factor kernel per cell and half-step, then one thread per line
template <typename T> hipError_t launch_epass_strag(const EParams<T> &P, int mode, hipStream_t st);
// FP32 with split-BF16 scans (Wh set or no next generation): thread per (cell, group of
// PBS_EPASS_LPT lines of an octet); deposits and records summed per group at line slot a = group
// (reduce over epass8_slots(NOCT) slots)
hipError_t launch_epass8(const EParams<float> &P, int mode, hipStream_t st);
// deposit slots per cell written by launch_epass8
__host__ __device__ inline int epass8_slots(int NOCT) { return NOCT * (8 / PBS_EPASS_LPT); }
template <typename T> hipError_t launch_tpass(const TParams<T> &P, hipStream_t st);
template <typename T> hipError_t launch_apass(const AParams<T> &P, int nth, long nstack, hipStream_t st);
template <typename T> hipError_t launch_qgemm(const QParams<T> &P, hipStream_t st);
template <typename T> hipError_t launch_fill(T *p, T v, long n, hipStream_t st);
// y = a y + b x elementwise
template <typename T> hipError_t launch_combine(T *y, const T *x, T a, T b, long n, hipStream_t st);
// edep_layer[pq] += sum over generations and the first nslot angular slots of dep
hipError_t launch_dose_reduce(double *edep_layer, const double *dep, int ngen, int NA, int nslot, long NLINE, int NP,
                              hipStream_t st);
hipError_t launch_dose_finalize(double *out, const double *edep, const double *rho, double vol, long n,
                                hipStream_t st);
template <typename T>
hipError_t launch_initial(T *psi0, const double *E1, const double *E2, const double *lat, long center_a, int G,
                          int NA, int NPB, int NP, hipStream_t st);

// split-BF16 source product: P2 as hi + lo; the scanned fluence as hi + lo (nprod = 3: three BF16
// products) or rounded once to BF16 (nprod = 2: two products); nprod = 1: one product of the
// column-compensated single-BF16 matrix (passed as Ahi) with the rounded scan.  Kernel kinds (same arithmetic, the
// same accumulation order per output): the scans read straight from global memory (default), or
// staged in LDS with 256- or 128-column blocks.
enum { QGEMM_GLOBAL_B = 0, QGEMM_LDS_256 = 1, QGEMM_LDS_128 = 2 };
hipError_t launch_qgemm_bf16s(const QParams<float> &P, const unsigned short *Ahi, const unsigned short *Alo, int Kp,
                              int nprod, hipStream_t st, int kind = QGEMM_GLOBAL_B);
hipError_t launch_apass_mfma32(const AParams<float> &P, const float *Ktab, long nstack, hipStream_t st);
hipError_t launch_apass_mfma16(const AParams<float> &P, const float *Ktab, long nstack, hipStream_t st);
// operand table of the MFMA angular pass for nth (16 or 32; 1024 floats, unused entries zero)
void apass_mfma_table(int nth, float *out1024);

bool apass_supported(int nth);

}  // namespace pbs
