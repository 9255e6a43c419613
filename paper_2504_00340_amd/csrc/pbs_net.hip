// Surrogate of the scattered generation: a 4-layer 3x3 convolutional network on the lateral grid of
// one depth slice, trained and evaluated by the kernels of this file.
//
//   layer 0   8 -> 32 channels, ReLU         (input: the solver's per-slice features, BF16)
//   layer 1  32 -> 32 channels, ReLU
//   layer 2  32 -> 32 channels, ReLU
//   layer 3  32 ->  1 channel,  linear       (output: FP32)
//
// Tensors are NHWC, BF16, channels innermost (8 or 32 stored channels).  Every convolution is an
// implicit GEMM on v_mfma_f32_16x16x32_bf16 with FP32 accumulation: M = 16 pixels of one image
// row, N = 16 output channels, K = 32 = (taps x input channels).  Weights are kept as FP32 master
// parameters (Adam state in FP32) and packed to BF16 operand tables after every update.  The
// weight gradient is reduced over pixels in two deterministic stages (per-block partials, then a
// fixed-order sum), so a training run is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pbs_net_internal.h"
#include "pbsplit.h"

namespace pbs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static const NetLayerDef kLayers[NET_LAYERS] = {
    // cin, cout, stored in, stored out (gradient), forward tile width
    {8, 32, 8, 32, 32},
    {32, 32, 32, 32, 32},
    {32, 32, 32, 32, 32},
    {32, 1, 32, 8, 16},
};

const NetLayerDef &net_layer(int l) { return kLayers[l]; }

size_t net_w_offset(int l)
{
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)kLayers[i].cout * kLayers[i].cin * 9 + kLayers[i].cout;
    return o;
}
size_t net_b_offset(int l) { return net_w_offset(l) + (size_t)kLayers[l].cout * kLayers[l].cin * 9; }
size_t net_param_count() { return net_w_offset(NET_LAYERS); }

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t net_packed_bytes()
{
    size_t o = 0;
    for (int l = 0; l < NET_LAYERS; ++l) {
        const NetLayerDef &d = kLayers[l];
        o = al256(o + (size_t)9 * d.coutp * d.cin_s * 2);
        if (l > 0) o = al256(o + (size_t)9 * d.cin_s * d.cout_s * 2);
        o = al256(o + (size_t)d.coutp * 4);
    }
    return o;
}

void net_carve(char *base, NetPacked &P)
{
    size_t o = 0;
    for (int l = 0; l < NET_LAYERS; ++l) {
        const NetLayerDef &d = kLayers[l];
        P.wf[l] = reinterpret_cast<__bf16 *>(base + o);
        o = al256(o + (size_t)9 * d.coutp * d.cin_s * 2);
        P.wb[l] = nullptr;
        if (l > 0) {
            P.wb[l] = reinterpret_cast<__bf16 *>(base + o);
            o = al256(o + (size_t)9 * d.cin_s * d.cout_s * 2);
        }
        P.bias[l] = reinterpret_cast<float *>(base + o);
        o = al256(o + (size_t)d.coutp * 4);
    }
}

// ------------------------------------------------------------------------------ convolution
constexpr int CV_TR = 4;       // image rows per block
constexpr int CV_WMAX = 64;    // widest image row: 4 waves x 16 pixels
enum { EPI_RELU = 0, EPI_LIN = 1, EPI_MASK = 2 };

// out[n][y][x][co] = sum_{tap, ci} in[n][y+ky-1][x+kx-1][ci] * w[tap][co][ci]   (zero outside the image)
//   EPI_RELU: + bias, ReLU, BF16 out [..][COUTP]
//   EPI_LIN : + bias of channel 0, FP32 out [..] (channel 0 only)
//   EPI_MASK: times [mask > 0] (mask: BF16 [..][COUTP]), BF16 out [..][COUTP]
// Block = CV_TR rows of one image; wave w owns pixels 16w .. 16w+15 of every row and all COUTP
// output channels.  The input rows (with a one-pixel halo) and the weights are staged in LDS.
template <int CIN, int COUTP, int EPI>
__global__ __launch_bounds__(256) void conv3x3_kernel(const __bf16 *__restrict__ in, const __bf16 *__restrict__ w,
                                                      const float *__restrict__ bias,
                                                      const __bf16 *__restrict__ mask, void *__restrict__ out, int H,
                                                      int Wd)
{
    constexpr int PXS = CIN + 8;   // LDS pixel stride (elements); keeps 16-byte alignment
    constexpr int WS = CIN + 8;
    constexpr int TPC = 32 / CIN;  // taps per MFMA step
    constexpr int NCH = (9 + TPC - 1) / TPC;
    constexpr int NJ = COUTP / 16;
    constexpr int C8 = CIN / 8;
    constexpr int LW = CV_WMAX + 2;
    __shared__ __attribute__((aligned(16))) __bf16 sin[(CV_TR + 2) * LW * PXS];
    __shared__ __attribute__((aligned(16))) __bf16 sw[9 * COUTP * WS];
    const int nrb = (H + CV_TR - 1) / CV_TR;
    const int n = blockIdx.x / nrb, y0 = (blockIdx.x % nrb) * CV_TR;
    const int tid = threadIdx.x;
    const int ncols = Wd + 2;
    const bf16x8 zero8 = {};
    for (int c = tid; c < (CV_TR + 2) * ncols * C8; c += 256) {
        const int c8 = c % C8, rc = c / C8, xx = rc % ncols, r = rc / ncols;
        const int y = y0 - 1 + r, x = xx - 1;
        bf16x8 v = zero8;
        if (y >= 0 && y < H && x >= 0 && x < Wd)
            v = *reinterpret_cast<const bf16x8 *>(in + (((long)n * H + y) * Wd + x) * CIN + 8 * c8);
        *reinterpret_cast<bf16x8 *>(&sin[(r * LW + xx) * PXS + 8 * c8]) = v;
    }
    for (int c = tid; c < 9 * COUTP * C8; c += 256) {
        const int c8 = c % C8, tco = c / C8;
        *reinterpret_cast<bf16x8 *>(&sw[tco * WS + 8 * c8]) =
            *reinterpret_cast<const bf16x8 *>(w + (long)tco * CIN + 8 * c8);
    }
    __syncthreads();
    const int wv = tid >> 6, l = tid & 63;
    const int x0 = wv * 16;
    if (x0 >= Wd) return;   // idle wave; no barrier follows
    f32x4 acc[CV_TR][NJ];
#pragma unroll
    for (int r = 0; r < CV_TR; ++r)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // operand k index of this lane: k = 8*(l/16) + i -> tap k / CIN, channel k % CIN
    const int kq = 8 * (l >> 4);
    const int tl = kq / CIN, ci0 = kq % CIN;
    const int px = x0 + (l & 15);
#pragma unroll
    for (int kc = 0; kc < NCH; ++kc) {
        const int t = kc * TPC + tl;
        const bool tv = t < 9;
        const int ky = tv ? t / 3 : 0, kx = tv ? t % 3 : 0;
        bf16x8 b[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            b[j] = tv ? *reinterpret_cast<const bf16x8 *>(&sw[(t * COUTP + 16 * j + (l & 15)) * WS + ci0]) : zero8;
#pragma unroll
        for (int r = 0; r < CV_TR; ++r) {
            bf16x8 a = zero8;
            if (tv && px < Wd) a = *reinterpret_cast<const bf16x8 *>(&sin[((r + ky) * LW + px + kx) * PXS + ci0]);
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[r][j], 0, 0, 0);
        }
    }
    // C layout: element q of lane l is (pixel 4*(l/16) + q, channel l % 16) of the 16 x 16 tile
#pragma unroll
    for (int r = 0; r < CV_TR; ++r) {
        const int y = y0 + r;
        if (y >= H) break;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int co = 16 * j + (l & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = x0 + 4 * (l >> 4) + q;
                if (p >= Wd) continue;
                const long pix = ((long)n * H + y) * Wd + p;
                float v = acc[r][j][q];
                if constexpr (EPI == EPI_RELU) {
                    v = fmaxf(v + bias[co], 0.f);
                    reinterpret_cast<__bf16 *>(out)[pix * COUTP + co] = (__bf16)v;
                } else if constexpr (EPI == EPI_LIN) {
                    if (co == 0) reinterpret_cast<float *>(out)[pix] = v + bias[0];
                } else {
                    const bool on = (float)mask[pix * COUTP + co] > 0.f;
                    reinterpret_cast<__bf16 *>(out)[pix * COUTP + co] = on ? (__bf16)v : (__bf16)0.f;
                }
            }
        }
    }
}

template <int CIN, int COUTP, int EPI>
static hipError_t conv3x3(const __bf16 *in, const __bf16 *w, const float *bias, const __bf16 *mask, void *out, int n,
                          int H, int Wd, hipStream_t st)
{
    const unsigned nb = (unsigned)((long)n * ((H + CV_TR - 1) / CV_TR));
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((conv3x3_kernel<CIN, COUTP, EPI>), dim3(nb), dim3(256), 0, st, in, w, bias, mask, out, H, Wd);
    return hipGetLastError();
}

// ------------------------------------------------------------------------- weight gradient
constexpr int WG_TR = 4;   // image rows per block

// Partial gradients over the WG_TR rows of one block:
//   part[blk][(tap*COP + co)*CIN + ci] = sum_px g[px][co] * in[px shifted by tap][ci]
//   part[blk][9*COP*CIN + co]          = sum_px g[px][co]
// MFMA: M = 16 output channels (A = g^T), N = 16 input channels (B = shifted input), K = 32 pixels.
template <int CIN, int COP>
__global__ __launch_bounds__(256) void wgrad_kernel(const __bf16 *__restrict__ in, const __bf16 *__restrict__ g,
                                                    float *__restrict__ part, int H, int Wd)
{
    constexpr int PXS = CIN + 2;   // odd word stride spreads the 2-byte column reads over banks
    constexpr int GS = COP + 2;
    constexpr int LW = CV_WMAX + 2;
    constexpr int MT = COP >= 16 ? COP / 16 : 1;
    constexpr int NT = CIN >= 16 ? CIN / 16 : 1;
    constexpr int NTILE = 9 * MT * NT;
    constexpr int TPW = (NTILE + 3) / 4;   // tiles per wave
    constexpr long PSZ = 9L * COP * CIN + COP;
    __shared__ __bf16 sin[(WG_TR + 2) * LW * PXS];
    __shared__ __bf16 sg[WG_TR * CV_WMAX * GS];
    __shared__ float red[256];
    const int nrb = (H + WG_TR - 1) / WG_TR;
    const int n = blockIdx.x / nrb, y0 = (blockIdx.x % nrb) * WG_TR;
    const int tid = threadIdx.x;
    const int ncols = Wd + 2;
    for (int c = tid; c < (WG_TR + 2) * ncols * CIN; c += 256) {
        const int ci = c % CIN, rc = c / CIN, xx = rc % ncols, r = rc / ncols;
        const int y = y0 - 1 + r, x = xx - 1;
        __bf16 v = (__bf16)0.f;
        if (y >= 0 && y < H && x >= 0 && x < Wd) v = in[(((long)n * H + y) * Wd + x) * CIN + ci];
        sin[(r * LW + xx) * PXS + ci] = v;
    }
    for (int c = tid; c < WG_TR * Wd * COP; c += 256) {
        const int co = c % COP, rx = c / COP, x = rx % Wd, r = rx / Wd;
        const int y = y0 + r;
        sg[(r * CV_WMAX + x) * GS + co] = y < H ? g[(((long)n * H + y) * Wd + x) * COP + co] : (__bf16)0.f;
    }
    __syncthreads();
    const int wv = tid >> 6, l = tid & 63;
    f32x4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nxc = (Wd + 31) / 32;
    for (int r = 0; r < WG_TR; ++r) {
        if (y0 + r >= H) break;
        for (int xc = 0; xc < nxc; ++xc) {
            const int xb = 32 * xc + 8 * (l >> 4);
            bf16x8 A[MT];
#pragma unroll
            for (int jm = 0; jm < MT; ++jm) {
                const int co = 16 * jm + (l & 15);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = xb + i;
                    A[jm][i] = (co < COP && x < Wd) ? sg[(r * CV_WMAX + x) * GS + co] : (__bf16)0.f;
                }
            }
#pragma unroll
            for (int ti = 0; ti < TPW; ++ti) {
                const int tile = wv + 4 * ti;
                if (tile >= NTILE) continue;
                const int tap = tile / (MT * NT), jm = (tile / NT) % MT, jn = tile % NT;
                const int ky = tap / 3, kx = tap % 3;
                const int ci = 16 * jn + (l & 15);
                bf16x8 B;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int x = xb + i;
                    B[i] = (ci < CIN && x < Wd) ? sin[((r + ky) * LW + x + kx) * PXS + ci] : (__bf16)0.f;
                }
                static_assert(MT <= 2, "at most two output-channel tiles");
                bf16x8 Aj = A[0];   // select without a dynamic register-array index
                if constexpr (MT > 1) {
                    if (jm == 1) Aj = A[1];
                }
                acc[ti] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aj, B, acc[ti], 0, 0, 0);
            }
        }
    }
    float *pb = part + (long)blockIdx.x * PSZ;
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti) {
        const int tile = wv + 4 * ti;
        if (tile >= NTILE) continue;
        const int tap = tile / (MT * NT), jm = (tile / NT) % MT, jn = tile % NT;
        const int ci = 16 * jn + (l & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int co = 16 * jm + 4 * (l >> 4) + q;
            if (co < COP && ci < CIN) pb[((long)tap * COP + co) * CIN + ci] = acc[ti][q];
        }
    }
    // bias partial: 256 / COP interleaved pixel subsets per channel, then a fixed-order sum
    constexpr int NS = 256 / COP;
    {
        const int co = tid % COP, sub = tid / COP;
        float s = 0.f;
        for (int rx = sub; rx < WG_TR * Wd; rx += NS) {
            const int r = rx / Wd, x = rx % Wd;
            s += (float)sg[(r * CV_WMAX + x) * GS + co];
        }
        red[tid] = s;
    }
    __syncthreads();
    if (tid < COP) {
        float s = 0.f;
        for (int k = 0; k < NS; ++k) s += red[k * COP + tid];
        pb[9L * COP * CIN + tid] = s;
    }
}

// grad (parameter order) = sum over blocks of the partials, real channels only
__global__ void wgrad_reduce_kernel(const float *__restrict__ part, long nblk, int CIN, int COP, int cin, int cout,
                                    float *__restrict__ gw, float *__restrict__ gb)
{
    const long PSZ = 9L * COP * CIN + COP;
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= PSZ) return;
    int co, ci = 0, tap = 0;
    const bool isb = e >= 9L * COP * CIN;
    if (isb) {
        co = (int)(e - 9L * COP * CIN);
        if (co >= cout) return;
    } else {
        tap = (int)(e / ((long)COP * CIN));
        co = (int)((e / CIN) % COP);
        ci = (int)(e % CIN);
        if (co >= cout || ci >= cin) return;
    }
    float s = 0.f;
    for (long b = 0; b < nblk; ++b) s += part[b * PSZ + e];
    if (isb)
        gb[co] = s;
    else
        gw[((long)co * cin + ci) * 9 + tap] = s;
}

template <int CIN, int COP>
static hipError_t wgrad(const __bf16 *in, const __bf16 *g, float *part, int n, int H, int Wd, int cin, int cout,
                        float *gw, float *gb, hipStream_t st)
{
    const long nblk = (long)n * ((H + WG_TR - 1) / WG_TR);
    const long PSZ = 9L * COP * CIN + COP;
    hipLaunchKernelGGL((wgrad_kernel<CIN, COP>), dim3((unsigned)nblk), dim3(256), 0, st, in, g, part, H, Wd);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((PSZ + 255) / 256)), dim3(256), 0, st, part, nblk, CIN,
                       COP, cin, cout, gw, gb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------- loss and optimiser
// Mean squared error over npx pixels: dy (channel 0 of 8) = 2 (y - t) / npx; per-block FP64 sums.
constexpr int LOSS_PER_THREAD = 8;
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ y, const float *__restrict__ t, long npx,
                                                  __bf16 *__restrict__ dy, double *__restrict__ lossp)
{
    __shared__ double red[256];
    const float sc = 2.0f / (float)npx;
    double s = 0.0;
    const long base = ((long)blockIdx.x * 256 + threadIdx.x) * LOSS_PER_THREAD;
    for (int i = 0; i < LOSS_PER_THREAD; ++i) {
        const long p = base + i;
        if (p >= npx) break;
        const float d = y[p] - t[p];
        s += (double)d * (double)d;
        bf16x8 v = {};
        v[0] = (__bf16)(sc * d);
        *reinterpret_cast<bf16x8 *>(dy + p * NET_CG) = v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lossp[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const double *__restrict__ lossp, long nb, long npx, double *__restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (long b = 0; b < nb; ++b) s += lossp[b];
    loss[0] = s / (double)npx;
}

__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, long n, float lr_t, float b1, float b2, float eps)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_t * mi / (sqrtf(vi) + eps);
}

// FP32 parameters of one layer (w [cout][cin][3][3], b [cout]) -> BF16 operand tables:
//   wf[tap][co][ci]      (co < coutp, ci < cin_s) forward
//   wb[tap'][ci][co]     (ci < cin_s, co < cout_s)   data gradient: tap' = 8 - tap (kernel flipped), channels swapped
__global__ void pack_layer_kernel(const float *__restrict__ w, const float *__restrict__ b, __bf16 *__restrict__ wf,
                                  __bf16 *__restrict__ wb, float *__restrict__ bias, int cin, int cout, int cin_s,
                                  int cout_s, int coutp)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e < 9L * coutp * cin_s) {
        const int tap = (int)(e / ((long)coutp * cin_s)), co = (int)((e / cin_s) % coutp), ci = (int)(e % cin_s);
        wf[e] = (co < cout && ci < cin) ? (__bf16)w[((long)co * cin + ci) * 9 + tap] : (__bf16)0.f;
    }
    if (wb && e < 9L * cin_s * cout_s) {
        const int tp = (int)(e / ((long)cin_s * cout_s)), ci = (int)((e / cout_s) % cin_s), co = (int)(e % cout_s);
        wb[e] = (co < cout && ci < cin) ? (__bf16)w[((long)co * cin + ci) * 9 + (8 - tp)] : (__bf16)0.f;
    }
    if (e < coutp) bias[e] = e < cout ? b[e] : 0.f;
}

hipError_t net_pack(const float *master, const NetPacked &P, hipStream_t st)
{
    for (int l = 0; l < NET_LAYERS; ++l) {
        const NetLayerDef &d = kLayers[l];
        long n = 9L * d.coutp * d.cin_s;
        if (l > 0) n = std::max(n, 9L * d.cin_s * d.cout_s);
        hipLaunchKernelGGL(pack_layer_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           master + net_w_offset(l), master + net_b_offset(l), P.wf[l], P.wb[l], P.bias[l], d.cin,
                           d.cout, d.cin_s, d.cout_s, d.coutp);
    }
    return hipGetLastError();
}

hipError_t net_forward(const NetPacked &P, const __bf16 *x, __bf16 *a1, __bf16 *a2, __bf16 *a3, float *y, int n,
                       int H, int Wd, hipStream_t st)
{
    hipError_t e;
    if ((e = conv3x3<8, 32, EPI_RELU>(x, P.wf[0], P.bias[0], nullptr, a1, n, H, Wd, st)) != hipSuccess) return e;
    if ((e = conv3x3<32, 32, EPI_RELU>(a1, P.wf[1], P.bias[1], nullptr, a2, n, H, Wd, st)) != hipSuccess) return e;
    if ((e = conv3x3<32, 32, EPI_RELU>(a2, P.wf[2], P.bias[2], nullptr, a3, n, H, Wd, st)) != hipSuccess) return e;
    return conv3x3<32, 16, EPI_LIN>(a3, P.wf[3], P.bias[3], nullptr, y, n, H, Wd, st);
}

// ----------------------------------------------------------------- per-slice surrogate features
__global__ __launch_bounds__(1024) void sur_scalars_kernel(const double *__restrict__ finj,
                                                           const double *__restrict__ fmn,
                                                           const double *__restrict__ edep,
                                                           const double *__restrict__ edep0, long n,
                                                           double *__restrict__ scal)
{
    __shared__ double r[5][1024];
    double mi = 0.0, mn = 0.0, si = 0.0, so = 0.0, s0 = 0.0;
    for (long i = threadIdx.x; i < n; i += 1024) {
        const double I = finj[i];
        mi = fmax(mi, I);
        mn = fmax(mn, fmn[i]);
        si += I;
        if (edep0) {
            so += edep[i] - edep0[i] + I;
            s0 += edep0[i];
        } else {
            s0 += edep[i];
        }
    }
    r[0][threadIdx.x] = mi;
    r[1][threadIdx.x] = mn;
    r[2][threadIdx.x] = si;
    r[3][threadIdx.x] = so;
    r[4][threadIdx.x] = s0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const int t = threadIdx.x;
            r[0][t] = fmax(r[0][t], r[0][t + w]);
            r[1][t] = fmax(r[1][t], r[1][t + w]);
            r[2][t] += r[2][t + w];
            r[3][t] += r[3][t + w];
            r[4][t] += r[4][t + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) scal[threadIdx.x] = r[threadIdx.x][0];
}

hipError_t sur_scalars(const double *finj, const double *fmn, const double *edep, const double *edep0, long n,
                       double *scal, hipStream_t st)
{
    hipLaunchKernelGGL(sur_scalars_kernel, dim3(1), dim3(1024), 0, st, finj, fmn, edep, edep0, n, scal);
    return hipGetLastError();
}

// one thread per lateral cell walks the layers in depth order (the filters are causal in depth)
__global__ void sur_features_kernel(SurFeatIn F, const double *__restrict__ scal, __bf16 *__restrict__ X,
                                    float *__restrict__ T)
{
    const int pq = blockIdx.x * 256 + threadIdx.x;
    if (pq >= F.NP) return;
    const double cb = scal[0] > 0.0 ? scal[0] : 1.0, cn = scal[1];
    const double icb = 1.0 / cb;
    double f[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < F.nz; ++s) {
        const long i = (long)s * F.NP + pq;
        const double I = F.finj[i], me = F.fme[i], mn = F.fmn[i], r = F.rho[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double a = exp(-r * F.dz / SUR_FILTER_L[j]);
            f[j] = a * f[j] + (1.0 - a) * I;
        }
        const double eb = (cn > 0.0 && mn > 1e-4 * cn) ? me / mn : 0.0;
        bf16x8 v = {};
        v[0] = (__bf16)(me * F.k0dz * icb);
        v[1] = (__bf16)r;
        v[2] = (__bf16)(I * icb);
        v[3] = (__bf16)(f[0] * icb);
        v[4] = (__bf16)(f[1] * icb);
        v[5] = (__bf16)(f[2] * icb);
        v[6] = (__bf16)(eb / SUR_EREF);
        v[7] = (__bf16)(f[3] * icb);
        *reinterpret_cast<bf16x8 *>(X + i * NET_CX) = v;
        if (T) T[i] = (float)((F.edep[i] - F.edep0[i] + I) * icb);
    }
}

hipError_t sur_features(const SurFeatIn &F, const double *scal, __bf16 *X, float *T, hipStream_t st)
{
    hipLaunchKernelGGL(sur_features_kernel, dim3((unsigned)((F.NP + 255) / 256)), dim3(256), 0, st, F, scal, X, T);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void sur_sum_kernel(const float *__restrict__ y, long n, double *__restrict__ out)
{
    __shared__ double r[1024];
    double s = 0.0;
    for (long i = threadIdx.x; i < n; i += 1024) s += (double)y[i];
    r[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = r[0];
}

hipError_t sur_sum(const float *y, long n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(sur_sum_kernel, dim3(1), dim3(1024), 0, st, y, n, out);
    return hipGetLastError();
}

__global__ void sur_combine_kernel(double *__restrict__ edep, const double *__restrict__ finj,
                                   const float *__restrict__ y, const double *__restrict__ scal, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const double cb = scal[0] > 0.0 ? scal[0] : 1.0;   // the feature scale
    if (i < n) edep[i] += cb * (double)y[i] - finj[i];
}

hipError_t sur_combine(double *edep, const double *finj, const float *y, const double *scal, long n, hipStream_t st)
{
    hipLaunchKernelGGL(sur_combine_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, edep, finj, y, scal,
                       n);
    return hipGetLastError();
}

__global__ void net_zero_kernel(float *__restrict__ p, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

}  // namespace pbs

// =================================================================================== C ABI
using namespace pbs;

struct pbs_net {
    int H = 0, W = 0, max_batch = 0;
    size_t npar = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0, total = 0;
    hipStream_t stream = nullptr;
    bool bound = false, have_params = false;
    long adam_t = 0;
    // workspace offsets
    size_t o_master = 0, o_m = 0, o_v = 0, o_grad = 0, o_packed = 0, o_a1 = 0, o_a2 = 0, o_a3 = 0, o_y = 0,
           o_dy = 0, o_ga = 0, o_gb = 0, o_part = 0, o_lossp = 0, o_loss = 0;
    NetPacked P;
    std::string err;

    template <typename T> T *at(size_t o) { return reinterpret_cast<T *>(ws + o); }
};

namespace {

pbs_status nfail(pbs_net *n, pbs_status s, const std::string &msg)
{
    if (n) n->err = msg;
    return s;
}

#define NHIP(n, expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return nfail((n), PBS_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

long loss_blocks(long npx) { return (npx + 256L * LOSS_PER_THREAD - 1) / (256L * LOSS_PER_THREAD); }

void net_layout(pbs_net *n)
{
    const size_t px = (size_t)n->max_batch * n->H * n->W;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al256(o + bytes);
        return at;
    };
    n->o_master = take(n->npar * 4);
    n->o_m = take(n->npar * 4);
    n->o_v = take(n->npar * 4);
    n->o_grad = take(n->npar * 4);
    n->o_packed = take(net_packed_bytes());
    n->o_a1 = take(px * NET_CH * 2);
    n->o_a2 = take(px * NET_CH * 2);
    n->o_a3 = take(px * NET_CH * 2);
    n->o_y = take(px * 4);
    n->o_dy = take(px * NET_CG * 2);
    n->o_ga = take(px * NET_CH * 2);
    n->o_gb = take(px * NET_CH * 2);
    const long nblk = (long)n->max_batch * ((n->H + WG_TR - 1) / WG_TR);
    size_t psz = 0;
    for (int l = 0; l < NET_LAYERS; ++l) {
        const NetLayerDef &d = kLayers[l];
        psz = std::max(psz, (size_t)9 * d.cout_s * d.cin_s + d.cout_s);
    }
    n->o_part = take((size_t)nblk * psz * 4);
    n->o_lossp = take((size_t)loss_blocks((long)px) * 8);
    n->o_loss = take(64);
    n->total = o;
}

// forward + loss + backward into the gradient buffer (parameter order); loss into o_loss
pbs_status net_grad(pbs_net *n, const __bf16 *x, const float *t, int nb)
{
    const int H = n->H, W = n->W;
    hipStream_t st = n->stream;
    __bf16 *a1 = n->at<__bf16>(n->o_a1), *a2 = n->at<__bf16>(n->o_a2), *a3 = n->at<__bf16>(n->o_a3);
    __bf16 *dy = n->at<__bf16>(n->o_dy), *ga = n->at<__bf16>(n->o_ga), *gb = n->at<__bf16>(n->o_gb);
    float *y = n->at<float>(n->o_y), *part = n->at<float>(n->o_part), *gr = n->at<float>(n->o_grad);
    NHIP(n, net_forward(n->P, x, a1, a2, a3, y, nb, H, W, st));
    const long npx = (long)nb * H * W;
    const long lb = loss_blocks(npx);
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)lb), dim3(256), 0, st, y, t, npx, dy, n->at<double>(n->o_lossp));
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(64), 0, st, n->at<double>(n->o_lossp), lb, npx,
                       n->at<double>(n->o_loss));
    NHIP(n, hipGetLastError());
    // layer 3 (linear, one output channel stored as 8)
    NHIP(n, (conv3x3<8, 32, EPI_MASK>(dy, n->P.wb[3], nullptr, a3, ga, nb, H, W, st)));
    NHIP(n, (wgrad<32, 8>(a3, dy, part, nb, H, W, 32, 1, gr + net_w_offset(3), gr + net_b_offset(3), st)));
    // layer 2
    NHIP(n, (conv3x3<32, 32, EPI_MASK>(ga, n->P.wb[2], nullptr, a2, gb, nb, H, W, st)));
    NHIP(n, (wgrad<32, 32>(a2, ga, part, nb, H, W, 32, 32, gr + net_w_offset(2), gr + net_b_offset(2), st)));
    // layer 1
    NHIP(n, (conv3x3<32, 32, EPI_MASK>(gb, n->P.wb[1], nullptr, a1, ga, nb, H, W, st)));
    NHIP(n, (wgrad<32, 32>(a1, gb, part, nb, H, W, 32, 32, gr + net_w_offset(1), gr + net_b_offset(1), st)));
    // layer 0
    NHIP(n, (wgrad<8, 32>(x, ga, part, nb, H, W, 8, 32, gr + net_w_offset(0), gr + net_b_offset(0), st)));
    return PBS_OK;
}

pbs_status net_check_call(pbs_net *n, const void *x, int nb)
{
    if (!n) return PBS_EINVAL;
    if (!n->bound) return nfail(n, PBS_ESTATE, "network not bound");
    if (!n->have_params) return nfail(n, PBS_ESTATE, "network parameters not set");
    if (!x) return nfail(n, PBS_EINVAL, "input is NULL");
    if (((uintptr_t)x & 15)) return nfail(n, PBS_EINVAL, "input must be 16-byte aligned");
    if (nb < 1 || nb > n->max_batch) return nfail(n, PBS_EINVAL, "batch must be in [1, max_batch]");
    return PBS_OK;
}

}  // namespace

extern "C" {

pbs_status pbs_net_param_count(size_t *count)
{
    if (!count) return PBS_EINVAL;
    *count = net_param_count();
    return PBS_OK;
}

pbs_status pbs_net_create(int H, int W, int max_batch, pbs_net **out)
{
    if (!out) return PBS_EINVAL;
    *out = nullptr;
    if (H < 1 || W < 1 || W > CV_WMAX || max_batch < 1) return PBS_EINVAL;
    if ((long)max_batch * H * W > (1L << 31) / NET_CH) return PBS_EINVAL;
    pbs_net *n = new (std::nothrow) pbs_net();
    if (!n) return PBS_ENOMEM;
    n->H = H;
    n->W = W;
    n->max_batch = max_batch;
    n->npar = net_param_count();
    net_layout(n);
    *out = n;
    return PBS_OK;
}

pbs_status pbs_net_workspace_bytes(const pbs_net *n, size_t *bytes)
{
    if (!n || !bytes) return PBS_EINVAL;
    *bytes = n->total;
    return PBS_OK;
}

pbs_status pbs_net_bind(pbs_net *n, void *ws, size_t bytes, void *stream)
{
    if (!n) return PBS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255)) return nfail(n, PBS_EINVAL, "workspace is NULL or not 256-byte aligned");
    if (bytes < n->total) return nfail(n, PBS_EINVAL, "workspace too small");
    n->ws = (char *)ws;
    n->ws_bytes = bytes;
    n->stream = (hipStream_t)stream;
    net_carve(n->ws + n->o_packed, n->P);
    n->bound = true;
    n->have_params = false;
    return PBS_OK;
}

pbs_status pbs_net_set_params(pbs_net *n, const float *params, size_t count)
{
    if (!n) return PBS_EINVAL;
    if (!n->bound) return nfail(n, PBS_ESTATE, "network not bound");
    if (!params || count != n->npar) return nfail(n, PBS_EINVAL, "parameter count mismatch");
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(params[i])) return nfail(n, PBS_EINVAL, "parameters must be finite");
    NHIP(n, hipMemcpyAsync(n->at<float>(n->o_master), params, count * 4, hipMemcpyHostToDevice, n->stream));
    const unsigned zb = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(net_zero_kernel, dim3(zb), dim3(256), 0, n->stream, n->at<float>(n->o_m), (long)count);
    hipLaunchKernelGGL(net_zero_kernel, dim3(zb), dim3(256), 0, n->stream, n->at<float>(n->o_v), (long)count);
    NHIP(n, hipGetLastError());
    NHIP(n, net_pack(n->at<float>(n->o_master), n->P, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    n->have_params = true;
    return PBS_OK;
}

pbs_status pbs_net_get_params(pbs_net *n, float *params, size_t count)
{
    if (!n) return PBS_EINVAL;
    if (!n->bound || !n->have_params) return nfail(n, PBS_ESTATE, "network parameters not set");
    if (!params || count != n->npar) return nfail(n, PBS_EINVAL, "parameter count mismatch");
    NHIP(n, hipMemcpyAsync(params, n->at<float>(n->o_master), count * 4, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    return PBS_OK;
}

pbs_status pbs_net_forward(pbs_net *n, const void *x, float *y, int nb)
{
    pbs_status r = net_check_call(n, x, nb);
    if (r != PBS_OK) return r;
    if (!y) return nfail(n, PBS_EINVAL, "output is NULL");
    NHIP(n, net_forward(n->P, (const __bf16 *)x, n->at<__bf16>(n->o_a1), n->at<__bf16>(n->o_a2),
                        n->at<__bf16>(n->o_a3), y, nb, n->H, n->W, n->stream));
    return PBS_OK;
}

pbs_status pbs_net_gradient(pbs_net *n, const void *x, const float *t, int nb, float *grad, size_t count, double *loss)
{
    pbs_status r = net_check_call(n, x, nb);
    if (r != PBS_OK) return r;
    if (!t || !grad || count != n->npar) return nfail(n, PBS_EINVAL, "target / gradient buffer invalid");
    if ((r = net_grad(n, (const __bf16 *)x, t, nb)) != PBS_OK) return r;
    NHIP(n, hipMemcpyAsync(grad, n->at<float>(n->o_grad), count * 4, hipMemcpyDeviceToHost, n->stream));
    double l = 0;
    NHIP(n, hipMemcpyAsync(&l, n->at<double>(n->o_loss), 8, hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    if (loss) *loss = l;
    return PBS_OK;
}

pbs_status pbs_net_train_step(pbs_net *n, const void *x, const float *t, int nb, double lr, double *loss_dev)
{
    pbs_status r = net_check_call(n, x, nb);
    if (r != PBS_OK) return r;
    if (!t) return nfail(n, PBS_EINVAL, "target is NULL");
    if (!(lr > 0) || !std::isfinite(lr)) return nfail(n, PBS_EINVAL, "learning rate must be finite and > 0");
    if ((r = net_grad(n, (const __bf16 *)x, t, nb)) != PBS_OK) return r;
    const double b1 = 0.9, b2 = 0.999;
    n->adam_t += 1;
    const double lr_t = lr * std::sqrt(1.0 - std::pow(b2, (double)n->adam_t)) / (1.0 - std::pow(b1, (double)n->adam_t));
    const long np = (long)n->npar;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, n->stream,
                       n->at<float>(n->o_master), n->at<float>(n->o_m), n->at<float>(n->o_v),
                       n->at<const float>(n->o_grad), np, (float)lr_t, (float)b1, (float)b2, 1e-8f);
    NHIP(n, hipGetLastError());
    NHIP(n, net_pack(n->at<float>(n->o_master), n->P, n->stream));
    if (loss_dev)
        NHIP(n, hipMemcpyAsync(loss_dev, n->at<double>(n->o_loss), 8, hipMemcpyDeviceToDevice, n->stream));
    return PBS_OK;
}

const char *pbs_net_last_error(const pbs_net *n) { return n ? n->err.c_str() : "null network"; }

void pbs_net_destroy(pbs_net *n) { delete n; }

}  // extern "C"
