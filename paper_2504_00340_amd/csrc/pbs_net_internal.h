// Internal declarations of the surrogate network and of the per-slice surrogate features.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pbs {

constexpr int NET_LAYERS = 4;
constexpr int NET_CX = 8;    // stored input channels (BF16) per pixel
constexpr int NET_CH = 32;   // hidden channels
constexpr int NET_CG = 8;    // stored channels of the output gradient
constexpr int SUR_NFEAT = 8; // feature channels the solver writes

struct NetLayerDef {
    int cin, cout;    // channels of the layer (parameters [cout][cin][3][3], bias [cout])
    int cin_s;        // stored channels of its input tensor
    int cout_s;       // stored channels of the gradient of its output
    int coutp;        // output channels of the forward MFMA tiles (multiple of 16)
};

// BF16 operand tables of all layers (device); carved from one block of net_packed_bytes()
struct NetPacked {
    __bf16 *wf[NET_LAYERS];    // [9][coutp][cin_s]
    __bf16 *wb[NET_LAYERS];    // [9][cin_s][cout_s], flipped taps (null for layer 0)
    float *bias[NET_LAYERS];   // [coutp]
};

const NetLayerDef &net_layer(int l);
size_t net_w_offset(int l);   // offsets in the flat FP32 parameter vector
size_t net_b_offset(int l);
size_t net_param_count();
size_t net_packed_bytes();
void net_carve(char *base, NetPacked &P);   // base: 256-byte aligned device memory
hipError_t net_pack(const float *master, const NetPacked &P, hipStream_t st);
// x [n][H][W][8] -> y [n][H][W]; a1, a2, a3: [n][H][W][32] activations (a3 may alias a1)
hipError_t net_forward(const NetPacked &P, const __bf16 *x, __bf16 *a1, __bf16 *a2, __bf16 *a3, float *y, int n,
                       int H, int W, hipStream_t st);

// ------------------------------------------------------------------ per-slice surrogate features
// Depth filters of the injected energy: F_j(s) = a F_j(s-1) + (1 - a) I(s), a = exp(-rho dz / L_j),
// with L_j in water-equivalent cm.
constexpr double SUR_FILTER_L[4] = {0.5, 2.0, 6.0, 15.0};
constexpr double SUR_EREF = 250.0;   // MeV, scale of the mean-energy channel

struct SurFeatIn {
    const double *finj;    // [nz][NP] energy injected into generation 1 (MeV per voxel layer)
    const double *fme;     // [nz][NP] energy moment of the primaries after the opening half-step
    const double *fmn;     // [nz][NP] number moment of the primaries after the opening half-step
    const double *rho;     // [nz][NP]
    const double *edep;    // [nz][NP] deposit of the whole march (target only)
    const double *edep0;   // [nz][NP] deposit of generation 0 (target only)
    int nz, NP;
    double dz, k0dz;       // step length; kappa0 * dz
};

// scal[0] = max finj, scal[1] = max fmn, scal[2] = sum finj, scal[3] = sum(edep - edep0 + finj)
// (0 without edep0), scal[4] = sum edep0 (sum edep without edep0); fixed-order reductions in one block
hipError_t sur_scalars(const double *finj, const double *fmn, const double *edep, const double *edep0, long n,
                       double *scal, hipStream_t st);
// X [nz][NP][8] BF16 features; T [nz][NP] FP32 targets (optional)
hipError_t sur_features(const SurFeatIn &F, const double *scal, __bf16 *X, float *T, hipStream_t st);
// out[0] = sum y (fixed order, FP64)
hipError_t sur_sum(const float *y, long n, double *out, hipStream_t st);
// edep += scal[0] * y - finj
hipError_t sur_combine(double *edep, const double *finj, const float *y, const double *scal, long n,
                       hipStream_t st);

}  // namespace pbs
