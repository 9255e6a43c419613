// libpbsplit batch planner: many pencil beams of one shape class marched together.
//
// Beams share the lateral grid, the angular grid and the number of generations; energy groups,
// depth steps and step length are per beam.  Beams are grouped into waves (longest first) that fit
// the caller's workspace; every wave's whole depth march is captured once into a HIP graph and
// launched as one graph launch.  Every kernel of a step covers all beams of the wave; blocks of
// beams that are done exit at once.  A small autotuner times bitwise-neutral launch variants
// (source-product tile width, transport waves per block, angular cells per block) on the first
// wave and keeps the fastest.  Tuning and capture happen once (pbs_batch_prepare, or the first run);
// later runs only set up each wave's state and replay its graph.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "pbs_common.h"
#include "pbs_ctx.h"
#include "pbsplit.h"

using namespace pbs;

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Slot {   // byte offsets of one beam's buffers inside the wave region
    size_t psi, Q, Wh, Wl, rho, rhod, dep, edep, tabf, tabd, ic, end;
};

}  // namespace

struct pbs_batch {
    int nb = 0;
    std::vector<pbs_grid> grids;
    std::vector<pbs_beam> beams;
    pbs_physics ph;
    std::vector<pbs_ctx *> ctx;   // host tables of every beam
    int nx = 0, ny = 0, nth = 0, m = 0, NA = 0, NP = 0, NPB = 0, NOCT = 0, ngen = 0, Kpb = 0, Mp = 0;
    long NLINE = 0;
    double dx = 0, dy = 0, dth = 0;
    int wave_cap = 0;
    std::vector<std::vector<int>> waves;
    std::vector<size_t> dose_off;   // doubles, per beam
    size_t o_shared = 0, o_beams = 0, o_dose = 0, o_wave = 0, total = 0;
    size_t sh_theta = 0, sh_lam = 0, sh_S = 0, sh_A = 0, sh_K = 0;   // byte offsets inside the shared block
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    // side stream of the captured march (each generation's T A T beside the energy chain)
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> ev_e, ev_tat;
    std::vector<char> pend;
    std::vector<std::vector<double>> rho;
    std::vector<char> have_rho;
    BatchTuning tune;
    bool tuned = false;
    // per wave: the whole march captured once (for the tuning chosen) and instantiated; replayed by every run
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    int state = 0;   // 0 created, 1 bound, 2 done
    std::string err;
};

namespace {

pbs_status bfail(pbs_batch *b, pbs_status st, const std::string &m)
{
    if (b) b->err = m;
    return st;
}

#define BHIP(b, expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return bfail((b), PBS_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

Slot slot_layout(const pbs_batch *b, int beam, size_t base)
{
    const int G = b->grids[beam].ng, nz = b->grids[beam].nz;
    Slot s;
    size_t o = base;
    s.psi = o;
    o = a256(o + (size_t)b->ngen * G * 2 * b->NLINE * 4);
    s.Q = o;
    if (b->ngen > 1) o = a256(o + (size_t)2 * G * b->NLINE * 4);
    const size_t wh = (size_t)2 * G * b->NPB * b->NOCT * PBS_PT * 8;   // elements of one of hi / lo
    s.Wh = o;
    if (b->ngen > 1) o = a256(o + wh * 2);
    s.Wl = o;
    if (b->ngen > 1) o = a256(o + wh * 2);
    s.rho = o;
    o = a256(o + (size_t)nz * b->NPB * PBS_PT * 4);
    s.rhod = o;
    o = a256(o + (size_t)nz * b->NP * 8);
    s.dep = o;
    o = a256(o + (size_t)2 * b->ngen * b->NLINE * 8);
    s.edep = o;
    o = a256(o + (size_t)nz * b->NP * 8);
    s.tabf = o;
    o = a256(o + (size_t)7 * G * 4);
    s.tabd = o;
    o = a256(o + (size_t)3 * G * 8);
    s.ic = o;
    o = a256(o + ((size_t)2 * G + b->NP) * 8);
    s.end = o;
    return s;
}

size_t wave_bytes(const pbs_batch *b, const std::vector<int> &w)
{
    size_t o = 0;
    for (int beam : w) o = slot_layout(b, beam, o).end;
    return o;
}

// Set up the resident state of one wave: tables, densities, zero fluence, initial condition.
pbs_status setup_wave(pbs_batch *b, const std::vector<int> &w, std::vector<BeamDev> &dev)
{
    dev.assign(w.size(), BeamDev());
    size_t o = 0;
    char *W = b->ws + b->o_wave;
    for (size_t j = 0; j < w.size(); ++j) {
        const int beam = w[j];
        const pbs_ctx *c = b->ctx[beam];
        const int G = c->G(), nz = b->grids[beam].nz;
        Slot s = slot_layout(b, beam, o);
        o = s.end;
        BeamDev &d = dev[j];
        d.psi = reinterpret_cast<float *>(W + s.psi);
        d.Q = reinterpret_cast<float *>(W + s.Q);
        d.Wh = reinterpret_cast<unsigned short *>(W + s.Wh);
        d.Wl = src_nprod(PBS_DEFAULT_SRC) == 3 ? reinterpret_cast<unsigned short *>(W + s.Wl) : nullptr;
        d.rho = reinterpret_cast<const float *>(W + s.rho);
        d.dep = reinterpret_cast<double *>(W + s.dep);
        d.edep = reinterpret_cast<double *>(W + s.edep);
        d.tabf = reinterpret_cast<const float *>(W + s.tabf);
        d.tabd = reinterpret_cast<const double *>(W + s.tabd);
        d.dBot = c->dBot;
        d.dz = (float)b->grids[beam].dz;
        d.thx = (float)(0.5 * (0.5 * c->g.dz) / c->dx);
        d.thy = (float)(0.5 * (0.5 * c->g.dz) / c->dy);
        d.G = G;
        d.nz = nz;
        // tables
        std::vector<float> tf((size_t)7 * G);
        for (int g = 0; g < G; ++g) {
            tf[g] = (float)c->Sm[g];
            tf[G + g] = (float)c->Sp[g];
            tf[2 * G + g] = (float)c->kappa[g];
            tf[3 * G + g] = (float)c->wc[g];
            tf[4 * G + g] = (float)c->wdec[g];
            tf[5 * G + g] = (float)c->invdE[g];
            tf[6 * G + g] = (float)c->sig_tr[g];
        }
        std::vector<double> td((size_t)3 * G);
        std::memcpy(td.data(), c->dA.data(), G * 8);
        std::memcpy(td.data() + G, c->dB.data(), G * 8);
        std::memcpy(td.data() + 2 * G, c->dInj.data(), G * 8);
        BHIP(b, hipMemcpyAsync(W + s.tabf, tf.data(), tf.size() * 4, hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(W + s.tabd, td.data(), td.size() * 8, hipMemcpyHostToDevice, b->stream));
        // densities (FP32, lateral tiles padded with 1) and FP64 copy for the dose
        std::vector<float> rf((size_t)nz * b->NPB * PBS_PT, 1.f);
        const std::vector<double> &rh = b->rho[beam];
        for (int z = 0; z < nz; ++z)
            for (int pq = 0; pq < b->NP; ++pq) rf[(size_t)z * b->NPB * PBS_PT + pq] = (float)rh[(size_t)z * b->NP + pq];
        BHIP(b, hipMemcpyAsync(W + s.rho, rf.data(), rf.size() * 4, hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(W + s.rhod, rh.data(), rh.size() * 8, hipMemcpyHostToDevice, b->stream));
        // zero fluence, scans (split-layout padding must stay zero) and dose
        BHIP(b, launch_fill<float>(d.psi, 0.f, (long)b->ngen * G * 2 * b->NLINE, b->stream));
        if (b->ngen > 1) BHIP(b, launch_fill<float>(reinterpret_cast<float *>(W + s.Wh), 0.f, (long)((s.rho - s.Wh) / 4), b->stream));
        BHIP(b, launch_fill<double>(d.edep, 0.0, (long)nz * b->NP, b->stream));
        // initial condition: eq:(bdy) projected, as for a single beam
        const pbs_beam &bm = b->beams[beam];
        auto ncdf = [](double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); };
        auto npdf = [](double x) { return std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI); };
        const pbs_grid &gr = b->grids[beam];
        std::vector<double> ic((size_t)2 * G + b->NP);
        double tx = 0, ty = 0, te = 0;
        std::vector<double> Lx(b->nx), Ly(b->ny);
        for (int p = 0; p < b->nx; ++p) {
            const double lo = -gr.x_half + p * b->dx;
            const double v = ncdf((lo + b->dx - bm.x0) / bm.sigma_x) - ncdf((lo - bm.x0) / bm.sigma_x);
            Lx[p] = v / b->dx;
            tx += v;
        }
        for (int q = 0; q < b->ny; ++q) {
            const double lo = -gr.y_half + q * b->dy;
            const double v = ncdf((lo + b->dy - bm.y0) / bm.sigma_y) - ncdf((lo - bm.y0) / bm.sigma_y);
            Ly[q] = v / b->dy;
            ty += v;
        }
        for (int g = 0; g < G; ++g) {
            const double lo = c->E_face[g], hi = c->E_face[g + 1], dE = hi - lo;
            const double za = (lo - bm.e0) / bm.sigma_e, zb = (hi - bm.e0) / bm.sigma_e;
            const double mass = ncdf(zb) - ncdf(za);
            const double mom = bm.sigma_e * (npdf(za) - npdf(zb)) + (bm.e0 - c->E_mid[g]) * mass;
            ic[g] = mass / dE;
            ic[G + g] = 6.0 * mom / (dE * dE);
            te += mass;
        }
        if (!(tx > 0 && ty > 0 && te > 0)) return bfail(b, PBS_EINVAL, "a beam does not overlap its grid");
        const double C = 1.0 / (tx * ty * te * b->dth * b->dth);
        for (int p = 0; p < b->nx; ++p)
            for (int q = 0; q < b->ny; ++q) ic[2 * G + (size_t)p * b->ny + q] = C * Lx[p] * Ly[q];
        BHIP(b, hipMemcpyAsync(W + s.ic, ic.data(), ic.size() * 8, hipMemcpyHostToDevice, b->stream));
        const double *icd = reinterpret_cast<const double *>(W + s.ic);
        const long center = (long)(b->m / 2) * b->m + b->m / 2;
        BHIP(b, launch_initial<float>(d.psi, icd, icd + G, icd + 2 * G, center, G, b->NA, b->NPB, b->NP, b->stream));
        BHIP(b, hipStreamSynchronize(b->stream));   // the host staging vectors of this beam end here
    }
    BHIP(b, hipMemcpyAsync(b->ws + b->o_beams, dev.data(), dev.size() * sizeof(BeamDev), hipMemcpyHostToDevice,
                           b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return PBS_OK;
}

BatchShape shape(const pbs_batch *b)
{
    BatchShape Sh;
    char *S = b->ws + b->o_shared;
    Sh.theta = reinterpret_cast<const float *>(S + b->sh_theta);
    Sh.lam = reinterpret_cast<const float *>(S + b->sh_lam);
    Sh.S = reinterpret_cast<const float *>(S + b->sh_S);
    Sh.K = reinterpret_cast<const float *>(S + b->sh_K);
    Sh.Ahi = reinterpret_cast<const unsigned short *>(S + b->sh_A);
    Sh.Alo = Sh.Ahi + (size_t)b->Mp * b->Kpb;
    if (src_nprod(PBS_DEFAULT_SRC) == 1) Sh.Ahi += (size_t)2 * b->Mp * b->Kpb;   // the compensated copy
    Sh.Kpb = b->Kpb;
    Sh.Mp = b->Mp;
    Sh.nprod = src_nprod(PBS_DEFAULT_SRC);
    Sh.nx = b->nx;
    Sh.ny = b->ny;
    Sh.nth = b->nth;
    Sh.m = b->m;
    Sh.NA = b->NA;
    Sh.NPB = b->NPB;
    Sh.NOCT = b->NOCT;
    Sh.ngen = b->ngen;
    Sh.NLINE = b->NLINE;
    Sh.dx = (float)b->dx;
    Sh.dy = (float)b->dy;
    Sh.scale = b->dth * b->dth * b->dx * b->dy;
    return Sh;
}

// time one fused step (s = 1) of the current wave with tuning t; returns ms or -1
float time_step(pbs_batch *b, int nw, int maxG, const BatchTuning &t)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    const BeamDev *bd = reinterpret_cast<const BeamDev *>(b->ws + b->o_beams);
    float best = -1.f;
    for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, b->stream);
        if (launch_batch_step(bd, nw, shape(b), 1, maxG, t, b->stream) != hipSuccess) break;
        (void)hipEventRecord(e1, b->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep == 1) best = ms;   // first repetition warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

pbs_status autotune(pbs_batch *b, int nw, int maxG)
{
    BatchTuning t = b->tune;
    t.max_nz = 2;
    const int gk[] = {QGEMM_GLOBAL_B, QGEMM_LDS_256, QGEMM_LDS_128}, wpb[] = {1, 2, 4}, pc[] = {8, 16, 32};
    auto pick = [&](int *field, const int *vals, int nv) {
        float bestms = 1e30f;
        int bestv = *field;
        for (int i = 0; i < nv; ++i) {
            if (field == &t.apass_pc && (size_t)b->NA * vals[i] * 4 > 64 * 1024) continue;
            *field = vals[i];
            const float ms = time_step(b, nw, maxG, t);
            if (ms > 0 && ms < bestms) {
                bestms = ms;
                bestv = vals[i];
            }
        }
        *field = bestv;
    };
    pick(&t.gemm_kind, gk, 3);
    pick(&t.tpass_wpb, wpb, 3);
    pick(&t.apass_pc, pc, 3);
    BHIP(b, hipGetLastError());
    b->tune.gemm_kind = t.gemm_kind;
    b->tune.tpass_wpb = t.tpass_wpb;
    b->tune.apass_pc = t.apass_pc;
    b->tuned = true;
    return PBS_OK;
}

int wave_max(const pbs_batch *b, const std::vector<int> &w, bool groups)
{
    int v = 0;
    for (int beam : w) v = std::max(v, groups ? b->grids[beam].ng : b->grids[beam].nz);
    return v;
}

// The whole march of wave wi captured into one graph and instantiated.  The kernels read the beam
// descriptors of the wave region at run time, so the graph serves every run (setup_wave writes them).
pbs_status capture_wave(pbs_batch *b, size_t wi)
{
    const std::vector<int> &w = b->waves[wi];
    const int maxG = wave_max(b, w, true), maxnz = wave_max(b, w, false);
    BatchTuning t = b->tune;
    t.max_nz = maxnz;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    const BeamDev *bd = reinterpret_cast<const BeamDev *>(b->ws + b->o_beams);
    const BatchShape Sh = shape(b);
    hipError_t le = hipSuccess;
    BatchSide sd{b->side, b->ev_e.data(), b->ev_tat.data(), b->pend.data()};
    for (int k = 0; k < b->ngen; ++k) b->pend[k] = 0;
    for (int s = 0; s <= maxnz && le == hipSuccess; ++s)
        le = launch_batch_step(bd, (int)w.size(), Sh, s, maxG, t, b->stream, &sd);
    // join the side stream before the capture ends
    for (int k = 0; k < b->ngen; ++k)
        if (b->pend[k]) {
            const hipError_t je = hipStreamWaitEvent(b->stream, b->ev_tat[k], 0);
            if (le == hipSuccess) le = je;
            b->pend[k] = 0;
        }
    const hipError_t ce = hipStreamEndCapture(b->stream, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bfail(b, PBS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return bfail(b, PBS_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    }
    b->graphs[wi] = graph;
    b->execs[wi] = exec;
    return PBS_OK;
}

void drop_graphs(pbs_batch *b)
{
    for (hipGraphExec_t e : b->execs)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : b->graphs)
        if (g) (void)hipGraphDestroy(g);
    b->execs.assign(b->waves.size(), nullptr);
    b->graphs.assign(b->waves.size(), nullptr);
}

// autotune on the first wave (once), then capture every wave not captured yet
pbs_status prepare(pbs_batch *b)
{
    if (b->execs.size() != b->waves.size()) drop_graphs(b);
    if (!b->tuned) {
        std::vector<BeamDev> dev;
        pbs_status r = setup_wave(b, b->waves[0], dev);
        if (r != PBS_OK) return r;
        if ((r = autotune(b, (int)b->waves[0].size(), wave_max(b, b->waves[0], true))) != PBS_OK) return r;
        drop_graphs(b);
    }
    for (size_t wi = 0; wi < b->waves.size(); ++wi)
        if (!b->execs[wi]) {
            const pbs_status r = capture_wave(b, wi);
            if (r != PBS_OK) return r;
        }
    return PBS_OK;
}

}  // namespace

// =================================================================================== C ABI
extern "C" {

pbs_status pbs_batch_create(const pbs_grid *grids, const pbs_beam *beams, int nbeams, const pbs_physics *phys,
                            int wave, pbs_batch **out)
{
    if (!out) return PBS_EINVAL;
    *out = nullptr;
    if (!grids || !beams || !phys || nbeams < 1 || wave < 0) return PBS_EINVAL;
    const pbs_grid &g0 = grids[0];
    for (int i = 0; i < nbeams; ++i) {
        const pbs_grid &g = grids[i];
        if (g.nx != g0.nx || g.ny != g0.ny || g.nth != g0.nth || g.ngen != g0.ngen || g.x_half != g0.x_half ||
            g.y_half != g0.y_half || g.th_half != g0.th_half)
            return PBS_EINVAL;   // one shape class per batch
    }
    if (g0.nth < 16) return PBS_EUNSUPPORTED;   // batched path: >= 128 angular unknowns (MFMA source product)
    if (phys->straggling || phys->nuc_bands > 1) return PBS_EUNSUPPORTED;   // single-beam path only
    pbs_batch *b = new (std::nothrow) pbs_batch();
    if (!b) return PBS_ENOMEM;
    b->nb = nbeams;
    b->grids.assign(grids, grids + nbeams);
    b->beams.assign(beams, beams + nbeams);
    b->ph = *phys;
    for (int i = 0; i < nbeams; ++i) {
        pbs_ctx *c = nullptr;
        const pbs_status r = pbs_create(&grids[i], phys, PBS_FP32, &c);
        if (r != PBS_OK) {
            for (pbs_ctx *x : b->ctx) pbs_destroy(x);
            delete b;
            return r;
        }
        b->ctx.push_back(c);
    }
    const pbs_ctx *c0 = b->ctx[0];
    b->nx = g0.nx;
    b->ny = g0.ny;
    b->nth = g0.nth;
    b->m = c0->m;
    b->NA = c0->NA;
    b->NP = c0->NP;
    b->NPB = c0->NPB;
    b->NOCT = c0->NOCT;
    b->ngen = g0.ngen;
    b->NLINE = c0->NLINE;
    b->Kpb = c0->Kpb;
    b->Mp = c0->Mp;
    b->dx = c0->dx;
    b->dy = c0->dy;
    b->dth = c0->dth;
    if (b->Kpb == 0) {
        pbs_batch_destroy(b);
        return PBS_EUNSUPPORTED;
    }
    // waves: longest beams first, wave beams resident at once
    std::vector<int> order(nbeams);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return grids[x].nz > grids[y].nz; });
    const int cap = wave > 0 ? wave : nbeams;
    b->wave_cap = cap;
    for (int i = 0; i < nbeams; i += cap)
        b->waves.emplace_back(order.begin() + i, order.begin() + std::min(nbeams, i + cap));
    // workspace: shared tables | beam descriptors | doses of all beams | largest wave
    size_t o = 0, sh = 0;
    b->sh_theta = sh;
    sh = a256(sh + (size_t)b->m * 4);
    b->sh_lam = sh;
    sh = a256(sh + (size_t)b->m * 4);
    b->sh_S = sh;
    sh = a256(sh + (size_t)b->m * b->m * 4);
    b->sh_A = sh;
    sh = a256(sh + (size_t)3 * b->Mp * b->Kpb * 2);
    b->sh_K = sh;
    sh = a256(sh + (size_t)1024 * 4);
    b->o_shared = o;
    o = a256(o + sh);
    b->o_beams = o;
    o = a256(o + (size_t)cap * sizeof(BeamDev));
    b->o_dose = o;
    size_t d = 0;
    for (int i = 0; i < nbeams; ++i) {
        b->dose_off.push_back(d);
        d += (size_t)grids[i].nz * b->NP;
    }
    o = a256(o + d * 8);
    b->o_wave = o;
    size_t wmax = 0;
    for (auto &w : b->waves) wmax = std::max(wmax, wave_bytes(b, w));
    b->total = a256(o + wmax);
    b->rho.assign(nbeams, {});
    b->have_rho.assign(nbeams, 0);
    while (b->tune.apass_pc > 8 && (size_t)b->NA * b->tune.apass_pc * 4 > 64 * 1024) b->tune.apass_pc /= 2;
    *out = b;
    return PBS_OK;
}

pbs_status pbs_batch_workspace_bytes(const pbs_batch *b, size_t *bytes)
{
    if (!b || !bytes) return PBS_EINVAL;
    *bytes = b->total;
    return PBS_OK;
}

pbs_status pbs_batch_bind(pbs_batch *b, void *ws, size_t bytes, void *stream)
{
    if (!b) return PBS_EINVAL;
    if (!ws || ((uintptr_t)ws & 255)) return bfail(b, PBS_EINVAL, "workspace is NULL or not 256-byte aligned");
    if (bytes < b->total) return bfail(b, PBS_EINVAL, "workspace too small");
    if (!stream) return bfail(b, PBS_EINVAL, "the batch needs a non-NULL stream (its march is captured into a graph)");
    b->ws = (char *)ws;
    b->stream = (hipStream_t)stream;
    if (!b->side) {
        BHIP(b, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        b->ev_e.assign(b->ngen, nullptr);
        b->ev_tat.assign(b->ngen, nullptr);
        b->pend.assign(b->ngen, 0);
        for (int k = 0; k < b->ngen; ++k) {
            BHIP(b, hipEventCreateWithFlags(&b->ev_e[k], hipEventDisableTiming));
            BHIP(b, hipEventCreateWithFlags(&b->ev_tat[k], hipEventDisableTiming));
        }
    }
    // shared angular tables and the split-BF16 nuclear angular transfer (identical for every beam)
    const pbs_ctx *c0 = b->ctx[0];
    std::vector<float> th(b->m), lam(b->m), S((size_t)b->m * b->m);
    for (int i = 0; i < b->m; ++i) {
        th[i] = (float)c0->theta[i];
        lam[i] = (float)c0->lam[i];
    }
    for (size_t i = 0; i < S.size(); ++i) S[i] = (float)c0->sinS[i];
    std::vector<unsigned short> A;
    transfer_table_bf16(c0->P2T, b->NA, b->Mp, b->Kpb, A);
    char *Sp = b->ws + b->o_shared;
    BHIP(b, hipMemcpyAsync(Sp + b->sh_theta, th.data(), th.size() * 4, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(Sp + b->sh_lam, lam.data(), lam.size() * 4, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(Sp + b->sh_S, S.data(), S.size() * 4, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(Sp + b->sh_A, A.data(), A.size() * 2, hipMemcpyHostToDevice, b->stream));
    std::vector<float> Kt(1024);
    apass_mfma_table(b->nth, Kt.data());
    BHIP(b, hipMemcpyAsync(Sp + b->sh_K, Kt.data(), Kt.size() * 4, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    b->state = 1;
    return PBS_OK;
}

pbs_status pbs_batch_set_phantom(pbs_batch *b, int beam, const double *rho, size_t n)
{
    if (!b) return PBS_EINVAL;
    if (beam < 0 || beam >= b->nb) return bfail(b, PBS_EINVAL, "beam index out of range");
    if (!rho || n != (size_t)b->grids[beam].nz * b->NP) return bfail(b, PBS_EINVAL, "phantom size must be nz*nx*ny");
    for (size_t i = 0; i < n; ++i)
        if (!(std::isfinite(rho[i]) && rho[i] > 0)) return bfail(b, PBS_EINVAL, "densities must be finite and > 0");
    b->rho[beam].assign(rho, rho + n);
    b->have_rho[beam] = 1;
    return PBS_OK;
}

pbs_status pbs_batch_prepare(pbs_batch *b)
{
    if (!b) return PBS_EINVAL;
    if (b->state < 1) return bfail(b, PBS_ESTATE, "batch_prepare before bind");
    for (int i = 0; i < b->nb; ++i)
        if (!b->have_rho[i]) return bfail(b, PBS_ESTATE, "a beam has no phantom");
    const pbs_status r = prepare(b);
    if (r != PBS_OK) return r;
    BHIP(b, hipStreamSynchronize(b->stream));
    return PBS_OK;
}

pbs_status pbs_batch_run(pbs_batch *b)
{
    if (!b) return PBS_EINVAL;
    if (b->state < 1) return bfail(b, PBS_ESTATE, "batch_run before bind");
    for (int i = 0; i < b->nb; ++i)
        if (!b->have_rho[i]) return bfail(b, PBS_ESTATE, "a beam has no phantom");
    pbs_status r = prepare(b);
    if (r != PBS_OK) return r;
    BHIP(b, launch_fill<double>(reinterpret_cast<double *>(b->ws + b->o_dose), 0.0,
                                (long)((b->o_wave - b->o_dose) / 8), b->stream));
    std::vector<BeamDev> dev;
    for (size_t wi = 0; wi < b->waves.size(); ++wi) {
        const std::vector<int> &w = b->waves[wi];
        if ((r = setup_wave(b, w, dev)) != PBS_OK) return r;
        const hipError_t re = hipGraphLaunch(b->execs[wi], b->stream);
        if (re != hipSuccess) return bfail(b, PBS_EDEVICE, std::string("graph launch: ") + hipGetErrorString(re));
        // dose of every beam of the wave
        size_t o = 0;
        for (int beam : w) {
            Slot s = slot_layout(b, beam, o);
            o = s.end;
            const pbs_grid &gr = b->grids[beam];
            const double vol = b->dx * b->dy * gr.dz;
            double *out = reinterpret_cast<double *>(b->ws + b->o_dose) + b->dose_off[beam];
            BHIP(b, launch_dose_finalize(out, reinterpret_cast<const double *>(b->ws + b->o_wave + s.edep),
                                         reinterpret_cast<const double *>(b->ws + b->o_wave + s.rhod), vol,
                                         (long)gr.nz * b->NP, b->stream));
        }
        // the next wave's set-up rewrites the wave region
        BHIP(b, hipStreamSynchronize(b->stream));
    }
    b->state = 2;
    return PBS_OK;
}

pbs_status pbs_batch_get_dose(pbs_batch *b, int beam, double *out, size_t n)
{
    if (!b) return PBS_EINVAL;
    if (b->state < 2) return bfail(b, PBS_ESTATE, "get_dose before batch_run");
    if (beam < 0 || beam >= b->nb) return bfail(b, PBS_EINVAL, "beam index out of range");
    if (!out || n != (size_t)b->grids[beam].nz * b->NP) return bfail(b, PBS_EINVAL, "dose buffer must hold nz*nx*ny");
    BHIP(b, hipMemcpyAsync(out, reinterpret_cast<double *>(b->ws + b->o_dose) + b->dose_off[beam], n * 8,
                           hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return PBS_OK;
}

pbs_status pbs_batch_tuning(const pbs_batch *b, int *out3)
{
    if (!b || !out3) return PBS_EINVAL;
    out3[0] = b->tune.gemm_kind;
    out3[1] = b->tune.tpass_wpb;
    out3[2] = b->tune.apass_pc;
    return PBS_OK;
}

const char *pbs_batch_last_error(const pbs_batch *b) { return b ? b->err.c_str() : "null batch"; }

void pbs_batch_destroy(pbs_batch *b)
{
    if (!b) return;
    if (b->ws) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graphs(b);
    for (hipEvent_t e : b->ev_e)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->ev_tat)
        if (e) (void)hipEventDestroy(e);
    if (b->side) (void)hipStreamDestroy(b->side);
    for (pbs_ctx *c : b->ctx) pbs_destroy(c);
    delete b;
}

}  // extern "C"
