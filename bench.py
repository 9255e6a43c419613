#!/usr/bin/env python3
"""Benchmark of the depth-splitting proton solver on one MI355X.

Headline workload: the heterogeneous case, the largest single-GPU configuration -- 180 MeV pencil beam
in a seeded layered water / bone / lung phantom with a half-plane bone insert and +-5 % smooth density
noise; lateral 96x96 cells over +-6 cm, 32x32 angular nodes over +-0.15 rad, 160 energy groups on
[0, 190] MeV, 400 depth steps over 26 cm, primary + 1 scattered generation; FP32 fluence, FP64 dose.
A step is one full depth step of every generation: the fused energy half-steps with the catastrophic
source, transport, angular diffusion, transport, dose reduction.  W untimed warm-up steps, then K
timed steps between stream synchronisations.

value = nx*ny*nth^2*G*(K+1) cell-updates per second (configured angular grid; the interior unknowns are
(nth-1)^2, also reported).  Kernel durations come from HIP events on the library's stream.  The
`roofline` entry is the dominant kernel of the timed region; `step_roofline` is the whole step against
the four-pass floor (64 B per interior cell-update).  Secondary legs: the 150 MeV water case (64x64,
128 groups, 4 generations), the batched plan (all 256 beams of the shared phantom), the learned
surrogate on held-out beams, and the FP64 oracle on a bounded sample of the headline workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_TFLOPS = 78.6     # 256 CU x 2.4 GHz x 64 lanes x 2 flop (packed FP32 not used)
FP32_MFMA_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2500.0   # dense
KINDS = ["epass", "tpass", "apass", "qgemm", "dose"]


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def algorithmic(grid, tsz=4, source="bf16x1"):
    """Algorithmic bytes (and flops of the source product) per launch of every kernel kind, with the
    energy scans W and the source Q counted in the form the mode stores them: FP32 contexts keep W as
    BF16 hi (+ lo in the three-product mode) and Q as BF16 in the single-product mode, FP32 otherwise."""
    nx, ny, nth, G, K1 = grid["nx"], grid["ny"], grid["nth"], grid["ng"], grid["ngen"]
    NA, NP = (nth - 1) ** 2, nx * ny
    lines = NA * NP
    split = tsz == 4 and source != "fp32" and NA >= 128
    wb = (4 if source == "bf16x3" else 2) if split else tsz      # bytes per scanned value
    qb = 2 if split and source == "bf16x1" else tsz               # bytes per source value
    # energy pass (fused pair): psi1, psi2 read + write (4 values per group and line), per line
    # two densities and two FP64 deposits; generation k>0 also reads the 2 source sums, k<K writes 2
    ep = []
    for k in range(K1):
        per = 4 * tsz + (2 * qb if k > 0 else 0) + (2 * wb if k + 1 < K1 else 0)
        ep.append(G * lines * per + lines * (2 * 8 + 2 * tsz))
    ep_bytes = sum(ep) / K1
    # T and A launch over all generations at once, or per generation (on the side stream) when one
    # generation has fewer than 1e8 phase-space cells
    per_launch = 1 if NP * NA * G < 100_000_000 else K1
    tp_bytes = per_launch * G * 2 * lines * 2 * tsz          # every plane read and written once
    ap_bytes = per_launch * G * 2 * lines * 2 * tsz + NP * tsz
    qg_flops = 2.0 * NA * NA * 2 * G * NP            # one source product (2 half-step sums) per generation
    qg_bytes = 2 * G * lines * (wb + qb) + NA * NA * (2 if split else tsz)
    return dict(epass=("bytes", ep_bytes), tpass=("bytes", tp_bytes), apass=("bytes", ap_bytes),
                qgemm=("flops", qg_flops, qg_bytes))


# kernel names of each kind at the two march workloads (as rocprofv3 reports them)
KIND_KERNEL = {
    "c3": {"tpass": "tpass_wide2_kernel", "apass": "apass_mfma32_kernel", "qgemm": "qgemm_bf16g_kernel<1>",
           "epass": "epass8_kernel<3, false, false, false>"},
    "c2": {"tpass": "tpass_affine_kernel<64>", "apass": "apass_mfma32_kernel", "qgemm": "qgemm_bf16g_kernel<1>",
           "epass": "epass8_kernel<3, false, false, false>"},
}
TRAFFIC_FILE = {"c3": "traffic_c3_hetero_fp32.md", "c2": "traffic_c2_water_fp32.md"}


def measured_traffic(tag, kind):
    """HBM bytes per dispatch of `kind` from the committed counter summary of this workload (FETCH_SIZE
    and WRITE_SIZE runs scaled by the copy calibration), or None when the kernels changed since then."""
    import hashlib

    if tag not in TRAFFIC_FILE or kind not in KIND_KERNEL[tag]:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE[tag])
    src = os.path.join(ROOT, "paper_2504_00340_amd", "csrc", "pbs_kernels.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if f"kernel_sha256_prefix {sha}" not in text:
        return None
    for line in text.split("```")[1].strip().splitlines():
        if line.startswith(KIND_KERNEL[tag][kind] + " "):
            return float(line.split()[-1])
    return None


def march(cfg, tag, precision, source, warmup, steps):
    """Time `steps` depth steps of one beam after `warmup` steps; per-kernel and step-level rooflines."""
    import torch

    from paper_2504_00340_amd import pbsplit as P

    g = cfg["grid"]
    if warmup + steps > g["nz"]:
        sys.exit(f"warmup + steps must be <= {g['nz']} depth steps")
    s = P.Solver(g, cfg["phys"], precision=precision, device="cuda:0")
    split = precision == "fp32" and source != "fp32"
    nprod = {"bf16x3": 3, "bf16x2": 2, "bf16x1": 1}.get(source, 2)
    if precision == "fp32":
        s.set_source_precision({"bf16x1": P.PBS_SRC_BF16X1, "bf16x2": P.PBS_SRC_BF16X2,
                                "bf16x3": P.PBS_SRC_BF16X3}.get(source, P.PBS_SRC_FP32))
    s.set_phantom(cfg["rho"])
    s.set_beam(cfg["beam"])
    s.step(warmup)
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    s.close()
    dt = (t1 - t0) / steps
    cells = g["nx"] * g["ny"] * g["nth"] ** 2 * g["ng"] * g["ngen"]
    interior = g["nx"] * g["ny"] * (g["nth"] - 1) ** 2 * g["ng"] * g["ngen"]
    log(f"{cfg['name']}: kernel totals over the timed region (ms, launches): "
        + ", ".join(f"{k} {v[0]:.1f}/{v[1]}" for k, v in prof.items()))
    tsz = 8 if precision == "fp64" else 4
    alg = algorithmic(g, tsz, source)
    kernels = {}
    for k, (ms, n) in prof.items():
        if n == 0:
            continue
        e = {"ms_per_step": ms / steps, "launches_per_step": n / steps, "avg_launch_ms": ms / n}
        if k in alg:
            b = alg[k][1] if alg[k][0] == "bytes" else alg[k][2]
            e["algorithmic_bytes_per_launch"] = b
            e["hbm_frac"] = b / (ms / n / 1e3) / 1e9 / HBM_PEAK_GBS
        kernels[k] = e
    dom = max((k for k in prof if k in alg and prof[k][1]), key=lambda k: prof[k][0])
    ms, n = prof[dom]
    avg_s = ms / max(n, 1) / 1e3
    ok = precision == "fp32" and source == "bf16x1"
    if alg[dom][0] == "bytes":
        achieved = alg[dom][1] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(tag, dom) if ok else None,
                "kernel": dom, "algorithmic_bytes_per_launch": alg[dom][1], "avg_launch_ms": avg_s * 1e3}
    else:
        mfma = precision == "fp32" and (g["nth"] - 1) ** 2 >= 128
        achieved = (nprod if split else 1) * alg[dom][1] / avg_s / 1e12
        peak = BF16_MFMA_TFLOPS if split else (FP32_MFMA_TFLOPS if mfma else FP32_VALU_TFLOPS)
        roof = {"bound": "mfma" if mfma else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "dtype": source if split else precision,
                "traffic": measured_traffic(tag, dom) if ok else None, "kernel": dom,
                "algorithmic_flops_per_launch": alg[dom][1], "avg_launch_ms": avg_s * 1e3}
    # the whole step against the four-pass floor: E pair, T, A, T each read and write both coefficients
    step_bytes = 4 * 2 * 2 * tsz * interior
    step_gbs = step_bytes / dt / 1e9
    return {"value": cells / dt, "ms_per_step": dt * 1e3, "interior_cell_updates_per_s": interior / dt,
            "beams_per_s": 1.0 / (dt * g["nz"]), "kernels": kernels, "roofline": roof,
            "step_roofline": {"bound": "hbm", "passes": 4, "bytes_per_cell_update": 4 * 2 * 2 * tsz,
                              "algorithmic_bytes_per_step": step_bytes, "achieved": step_gbs,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS}}


def cpu_baseline(cfg):
    """FP64 oracle on a bounded sample of the headline workload: the same physics and angular / energy
    grids on a small lateral window of the same cell size, one depth step, all generations; once with
    every host thread (16x16 window) and once with one thread (4x4 window)."""
    import numpy as np

    from oracle import oracle as O

    out = {}
    cores = O.max_threads()
    for label, n, threads in (("all", 16, cores), ("one", 4, 1)):
        dx = 2 * cfg["grid"]["x_half"] / cfg["grid"]["nx"]
        g = dict(cfg["grid"], nx=n, ny=n, x_half=n * dx / 2, y_half=n * dx / 2, nz=1)
        O.set_threads(threads)
        o = O.Oracle(g, cfg["phys"])
        st = o.initial(cfg["beam"])
        t0 = time.perf_counter()
        o.run(cfg["beam"], np.ones((1, n, n)), state=st)
        dt = time.perf_counter() - t0
        cells = g["nx"] * g["ny"] * g["nth"] ** 2 * g["ng"] * g["ngen"]
        out[label] = (cells / dt, threads, f"1 depth step of the workload on a {n}x{n} lateral window "
                                           f"(same cells, angles, groups, {g['ngen']} generations): {dt:.2f} s")
    O.set_threads(cores)
    return {"value": out["all"][0], "unit": "cell-updates/s", "cores": out["all"][1], "kind": "oracle",
            "sample": out["all"][2], "value_1_thread": out["one"][0], "sample_1_thread": out["one"][2]}


def batched(nbeams, wave, nsingle):
    """The batched plan: `nbeams` uneven beams (energies, groups, depths) on 32x32 windows of a shared
    128x128x400 phantom, one graph launch per wave (waves of `wave` beams), against the single-beam path
    timed on the first `nsingle` beams and extrapolated by cell-updates."""
    import torch

    from paper_2504_00340_amd import inputs as I
    from paper_2504_00340_amd.pbsplit import Batch, Solver

    cfg = I.config4(seed=0, nbeams=nbeams)
    beams, ph = cfg["beams"], cfg["phys"]

    def cells(bs):
        return sum(b["grid"]["nx"] * b["grid"]["ny"] * b["grid"]["nth"] ** 2 * b["grid"]["ng"] * b["grid"]["ngen"]
                   * b["grid"]["nz"] for b in bs)

    sub = beams[:nsingle]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in sub:
        s = Solver(b["grid"], ph, precision="fp32")
        s.set_phantom(b["rho"])
        s.set_beam(b["beam"])
        s.run()
        s.dose()
        s.close()
    torch.cuda.synchronize()
    t_sub = time.perf_counter() - t0
    torch.cuda.empty_cache()
    log(f"batched leg: single-beam path on {nsingle} beams {t_sub:.1f} s")
    bt = Batch(beams, ph, wave=wave)
    t0 = time.perf_counter()
    bt.prepare()                # autotuner + one graph capture per wave (not timed)
    t_prep = time.perf_counter() - t0
    log(f"batched leg: prepared {nbeams} beams in waves of {wave} ({t_prep:.1f} s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    tuning = bt.tuning()
    bt.close()
    torch.cuda.empty_cache()
    cs, ca = cells(sub), cells(beams)
    t_single_est = t_sub * ca / cs
    return {"workload": f"{cfg['name']}: all {nbeams} beams, E in "
                        f"[{min(b['beam']['e0'] for b in beams):.0f}, {max(b['beam']['e0'] for b in beams):.0f}] MeV, "
                        f"G {min(b['grid']['ng'] for b in beams)}-{max(b['grid']['ng'] for b in beams)}, "
                        f"{min(b['grid']['nz'] for b in beams)}-{max(b['grid']['nz'] for b in beams)} steps, "
                        f"32x32 cells, 16x16 angles, 2 generations",
            "beams": nbeams, "wave": wave, "seconds": t_batch, "beams_per_s": nbeams / t_batch,
            "cell_updates_per_s": ca / t_batch,
            "beams_per_s_single_beam_path": nbeams / t_single_est,
            "single_beam_path": f"extrapolated from the first {nsingle} beams ({t_sub:.2f} s, {cs:.3e} of "
                                f"{ca:.3e} cell-updates)",
            "speedup": t_single_est / t_batch, "prepare_s": t_prep, "tuning": tuning}


def surrogate(nseeds, tol=1e-2):
    """Held-out beams of the surrogate workload: the plain K = 1 march against the surrogate of generation 1
    (weights shipped with the package; residual test with fallback to the plain march)."""
    import numpy as np
    import torch

    from paper_2504_00340_amd import inputs as I
    from paper_2504_00340_amd.pbsplit import Solver, surrogate_weights

    blob = surrogate_weights()
    t = {"plain": 0.0, "surrogate": 0.0}
    rows = []
    for seed in range(100_000, 100_000 + nseeds):
        c = I.config5(seed)
        dose = {}
        for mode in ("plain", "surrogate"):
            s = Solver(c["grid"], c["phys"], "fp32", surrogate=blob if mode == "surrogate" else None,
                       residual_tol=tol)
            s.set_phantom(c["rho"])
            s.set_beam(c["beam"])
            s.run()                          # warm-up beam
            s.set_beam(c["beam"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run()
            rep = s.surrogate_report() if mode == "surrogate" else None
            torch.cuda.synchronize()
            t[mode] += time.perf_counter() - t0
            dose[mode] = s.dose()
            s.close()
        err = float(np.linalg.norm(dose["surrogate"] - dose["plain"]) / np.linalg.norm(dose["plain"]))
        rows.append({"seed": seed, "e0": round(c["beam"]["e0"], 2), "rel_l2_dose_error": err,
                     "residual": rep["residual"], "fallback": bool(rep["fallback"])})
    return {"workload": f"surrogate held-out seeds 100000-{100_000 + nseeds - 1}: 64x64 cells, 16x16 angles, "
                        f"96 groups, 300 steps, K = 1, FP32",
            "beams_per_s_plain": nseeds / t["plain"], "beams_per_s_surrogate": nseeds / t["surrogate"],
            "speedup": t["plain"] / t["surrogate"], "tolerance": tol,
            "max_rel_l2_dose_error": max(r["rel_l2_dose_error"] for r in rows),
            "fallbacks": sum(r["fallback"] for r in rows), "beams": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2"],
                    help="headline march: c3 (heterogeneous 96x96, 160 groups, K = 1) or c2 (150 MeV water)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--source", default="bf16x1", choices=["bf16x1", "bf16x2", "bf16x3", "fp32"],
                    help="arithmetic of the angular source product (FP32 contexts)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the second march workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-beams", type=int, default=256,
                    help="beams of the batched plan (0 = skip)")
    ap.add_argument("--batch-wave", type=int, default=128, help="beams resident per wave of the batch")
    ap.add_argument("--single-beams", type=int, default=16,
                    help="beams run through the single-beam path for the batched comparison")
    ap.add_argument("--surrogate-beams", type=int, default=4,
                    help="held-out beams for the surrogate leg (0 = skip)")
    ap.add_argument("--only", default=None, choices=["march", "batched", "surrogate"],
                    help="run one leg only (for profiling); prints that leg's JSON object")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the multi-GPU sharding is a design note, "
              "not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_00340_amd import inputs as I

    if args.only == "batched":
        print(json.dumps({"batched": batched(args.batched_beams, args.batch_wave, args.single_beams)}))
        return
    if args.only == "surrogate":
        print(json.dumps({"surrogate": surrogate(max(1, args.surrogate_beams))}))
        return
    cfg = I.config3(0) if args.workload == "c3" else I.config2("water")
    g = cfg["grid"]
    log(f"{cfg['name']} {args.precision}, warmup {args.warmup}, steps {args.steps}")
    head = march(cfg, args.workload, args.precision, args.source, args.warmup, args.steps)
    torch.cuda.empty_cache()
    split = args.precision == "fp32" and args.source != "fp32"
    desc = (f"{g['nx']}x{g['ny']} lateral x {g['nth']}x{g['nth']} angles x {g['ng']} groups x {g['ngen']} "
            f"generations, {g['nz']} depth steps")
    out = {
        "metric": "phase-space cell-updates/s per z-step",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: {desc}", "steps_per_beam": g["nz"], "precision": args.precision,
                   "source_product": args.source if split else args.precision},
        "interior_cell_updates_per_s": head["interior_cell_updates_per_s"],
        "beams_per_s": head["beams_per_s"],
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "step_roofline": head["step_roofline"],
    }
    if args.calibrate_copy:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n}
        del src, dst
        torch.cuda.empty_cache()
    if args.only == "march":
        print(json.dumps(out))
        return
    if not args.no_secondary:
        other = "c2" if args.workload == "c3" else "c3"
        c2 = I.config2("water") if other == "c2" else I.config3(0)
        g2 = c2["grid"]
        log(f"secondary march {c2['name']}")
        sec = march(c2, other, args.precision, args.source, args.warmup, args.steps)
        torch.cuda.empty_cache()
        out["secondary"] = {"workload": f"{c2['name']}: {g2['nx']}x{g2['ny']} lateral x {g2['nth']}x{g2['nth']} "
                                        f"angles x {g2['ng']} groups x {g2['ngen']} generations, {g2['nz']} steps",
                            **sec}
    if args.batched_beams > 0:
        log(f"batched leg, {args.batched_beams} beams")
        out["batched"] = batched(args.batched_beams, args.batch_wave, args.single_beams)
    if args.surrogate_beams > 0:
        log(f"surrogate leg, {args.surrogate_beams} held-out beams")
        out["surrogate"] = surrogate(args.surrogate_beams)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
