// Host-side context of one beam (shared by the single-beam ABI and the batch planner).
#pragma once
#include <string>
#include <utility>
#include <vector>

#include "pbs_common.h"
#include "pbsplit.h"

enum { ST_CREATED = 0, ST_BOUND = 1, ST_PHANTOM = 2, ST_BEAM = 3 };

// source-product arithmetic of FP32 contexts with >= 128 angular unknowns (and of every batch)
constexpr int PBS_DEFAULT_SRC = PBS_SRC_BF16X1;
inline int src_nprod(int mode) { return mode == PBS_SRC_BF16X1 ? 1 : mode == PBS_SRC_BF16X2 ? 2 : 3; }

struct pbs_ctx;
namespace pbs {
// bind a workspace and a stream (uploads the tables); with_side creates the two-stream march's stream and events
pbs_status bind_workspace(pbs_ctx *c, char *ws, size_t bytes, hipStream_t stream, bool with_side);
// record an error on the context and return st
pbs_status ctx_fail(pbs_ctx *c, pbs_status st, const char *msg);
// true when another context has been bound to the static scratch of c's device since c was
bool static_lost(const pbs_ctx *c);
// split-BF16 transfer matrix [3][Mp][Kpb]: hi, lo, and a column-compensated single-BF16 copy
void transfer_table_bf16(const std::vector<double> &P2T, int NA, int Mp, int Kpb, std::vector<unsigned short> &out);
}  // namespace pbs

struct pbs_ctx {
    pbs_grid g;
    pbs_physics ph;
    int prec = PBS_FP32;
    int tsz = 4;                          // sizeof(T)
    int m = 0, NA = 0, NP = 0, NPB = 0, NPpad = 0;
    long NLINE = 0;
    double dx = 0, dy = 0, dth = 0;
    // host tables (FP64)
    std::vector<double> E_face, E_mid, dE, S_face, sig_tr, kappa, Sm, Sp, wc, wdec, invdE, dA, dB, dInj, theta, sinS,
        lam, P2T;
    double dBot = 0;
    // nuclear bands (App. A.4): NB angular laws P2T [NB][NA][NA], band of every group, per-band decays of the
    // energy scan [NB][G]
    int NB = 1;
    std::vector<int> band;
    std::vector<double> wdecb;
    // straggling: rho-free 2x2 blocks of the energy operator per group [G][12] = Lo (to g-1), Di, Up (to g+1),
    // row-major, and the deposit functional's weights of psi1, psi2 [G] (the whole operator)
    bool strag = false;
    std::vector<double> blk, dA2, dB2;
    // splitting in depth: 2 Strang steps, 4 Richardson-extrapolated Strang steps (two state copies and two
    // scratch deposit rows edep(nz), edep(nz + 1))
    int order = 2;
    size_t o_x0 = 0, o_xA = 0;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    // side stream of the depth march: generation k's T A T runs there while the main stream continues
    // with the source product and the later generations' energy passes
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> ev_e, ev_tat;   // per generation: energy pass done / T A T done
    std::vector<char> tat_pend;             // T A T issued and not yet waited for by the main stream
    int sched = 0;                          // PBS_SCHED_*
    size_t o_psi = 0, o_W = 0, o_Q = 0, o_dep = 0, o_edep = 0, o_dout = 0, o_rhoT = 0, o_rhoD = 0, o_tabT = 0,
           o_tabD = 0, total = 0;
    // table offsets (elements) inside the T and double table blocks
    size_t t_Sm, t_Sp, t_kap, t_wc, t_wdec, t_invdE, t_sig, t_theta, t_S, t_lam, t_P2T, t_P2p, t_K32, t_wdecb, t_blk,
        t_count;
    size_t o_band = 0, o_sfac = 0;   // band indices [G] (int); straggling factors [2][G][8][NPpad] (T)
    int Kp = 0, Mp = 0;           // padded source product (MFMA path, FP32 with NA >= 128)
    int Kpb = 0;                  // k padding of the split-BF16 operand tables
    int NOCT = 0;                 // source-node octets of the split-BF16 W layout
    size_t Wb_half = 0;           // elements of one of the hi / lo arrays
    int src_mode = PBS_SRC_FP32;
    size_t o_bf = 0;
    size_t d_A, d_B, d_Inj, d_E1, d_E2, d_lat, d_A2, d_B2, d_count;
    int state = ST_CREATED;
    int step = 0;
    // bound to the static scratch of device static_dev (-1: caller workspace) when the scratch's owner
    // count of that device was static_epoch
    int static_dev = -1;
    unsigned long long static_epoch = 0;
    bool closed = false;
    std::vector<double> rho_host;
    std::string err;
    // kernel timing (diagnostics)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_pairs;   // (kind, index of the start event)

    // surrogate of the scattered generation
    int sur = 0;                  // 0 off, 1 recording, 2 surrogate with fallback
    double sur_tol = 0, sur_leak[3] = {0, 0, 0};
    std::vector<float> sur_params;
    int kact = 0;                 // generations marched (g.ngen, or 1 while the surrogate runs)
    bool feat_on = false;         // record the per-slice surrogate data in the march
    double sur_rep[10] = {};
    pbs_beam beam{};
    size_t o_fl = 0, o_frec = 0, o_scal = 0, o_sx = 0, o_sy = 0, o_sa = 0, o_sb = 0, o_spk = 0, o_smaster = 0;
    size_t d_wmom = 0;

    double *fline(int i) { return reinterpret_cast<double *>(ws + o_fl) + (size_t)i * NLINE; }
    // records [4][nz][NP]: 0 injected energy, 1 energy moment, 2 number moment, 3 generation-0 deposit
    double *frec(int i, int s) { return reinterpret_cast<double *>(ws + o_frec) + ((size_t)i * g.nz + s) * NP; }
    double *scal() { return reinterpret_cast<double *>(ws + o_scal); }

    template <typename T> T *psi(int k) { return reinterpret_cast<T *>(ws + o_psi) + (size_t)k * G() * 2 * NLINE; }
    template <typename T> T *W() { return reinterpret_cast<T *>(ws + o_W); }
    template <typename T> T *Q() { return reinterpret_cast<T *>(ws + o_Q); }
    template <typename T> T *tabT() { return reinterpret_cast<T *>(ws + o_tabT); }
    template <typename T> T *rhoT(int s) { return reinterpret_cast<T *>(ws + o_rhoT) + (size_t)s * NPpad; }
    double *tabD() { return reinterpret_cast<double *>(ws + o_tabD); }
    double *dep(int half, int k) { return reinterpret_cast<double *>(ws + o_dep) + ((size_t)half * g.ngen + k) * NLINE; }
    double *edep(int s) { return reinterpret_cast<double *>(ws + o_edep) + (size_t)s * NP; }
    double *dout() { return reinterpret_cast<double *>(ws + o_dout); }
    double *rhoD() { return reinterpret_cast<double *>(ws + o_rhoD); }
    int G() const { return g.ng; }
};
