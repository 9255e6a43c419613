#!/usr/bin/env python3
"""Benchmark of the depth-splitting proton solver on one MI355X.

Workload (default): 150 MeV pencil beam in water, lateral 64x64 cells over +-4 cm, 32x32 angular
nodes over +-0.15 rad, 128 energy groups on [0,160] MeV, 300 depth steps over 18 cm, primary + 3
scattered generations, FP32 fluence with FP64 dose.  A step is one full depth step of every
generation: fused energy half-steps with the catastrophic source, transport, angular diffusion,
transport, dose reduction.  W untimed warm-up steps, then K timed steps between stream
synchronisations.

value = nx*ny*nth^2*G*(K+1) cell-updates per second (configured angular grid; the interior
unknowns are (nth-1)^2 -- also reported).  The roofline entry is the dominant kernel of the timed
region, its duration measured with HIP events on the library's stream; cpu_baseline is the FP64
oracle on a bounded sample of the same workload.
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


def algorithmic(grid, tsz=4):
    """Algorithmic bytes / flops per launch of every kernel kind for one depth step."""
    nx, ny, nth, G, K1 = grid["nx"], grid["ny"], grid["nth"], grid["ng"], grid["ngen"]
    NA, NP = (nth - 1) ** 2, nx * ny
    lines = NA * NP
    # energy pass (fused pair): psi1, psi2 read + write (4 values per group and line), per line
    # two densities and two FP64 deposits; generation k>0 also reads the 2 source sums, k<K writes 2
    ep = []
    for k in range(K1):
        per = 4 * tsz + (2 * tsz if k > 0 else 0) + (2 * tsz if k + 1 < K1 else 0)
        ep.append(G * lines * per + lines * (2 * 8 + 2 * tsz))
    ep_bytes = sum(ep) / K1
    # T and A launch over all generations at once, or per generation (on the side stream) when one
    # generation has fewer than 1e8 phase-space cells
    per_launch = 1 if NP * NA * G < 100_000_000 else K1
    tp_bytes = per_launch * G * 2 * lines * 2 * tsz          # every plane read and written once
    ap_bytes = per_launch * G * 2 * lines * 2 * tsz + NP * tsz
    qg_flops = 2.0 * NA * NA * 2 * G * NP            # one source product (2 half-step sums) per generation
    qg_bytes = 2 * G * lines * 2 * tsz + NA * NA * tsz
    return dict(epass=("bytes", ep_bytes), tpass=("bytes", tp_bytes), apass=("bytes", ap_bytes),
                qgemm=("flops", qg_flops, qg_bytes))


KIND_KERNEL = {"tpass": "tpass_affine_kernel<64>", "apass": "apass_mfma32_kernel", "qgemm": "qgemm_bf16g_kernel<1>",
               "epass": "epass8_kernel<3, false, false>"}


def measured_traffic(kind):
    """HBM bytes per dispatch of `kind` from the committed counter summary (FETCH_SIZE/WRITE_SIZE runs of
    this workload, scaled by the copy calibration), or None when the kernels changed since then."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_c2_water_fp32.md")
    src = os.path.join(ROOT, "paper_2504_00340_amd", "csrc", "pbs_kernels.hip")
    if not os.path.exists(path) or kind not in KIND_KERNEL:
        return None
    text = open(path).read()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if f"kernel_sha256_prefix {sha}" not in text:
        return None
    for line in text.split("```")[1].strip().splitlines():
        if line.startswith(KIND_KERNEL[kind] + " "):
            return float(line.split()[-1])
    return None


def cpu_baseline(cfg):
    """FP64 oracle on a bounded sample: the same physics and angular/energy grid on a 12x12 lateral
    window (same cell size), 1 depth step, all generations."""
    import numpy as np

    from oracle import oracle as O

    n = 12
    g = dict(cfg["grid"], nx=n, ny=n, x_half=n * 0.0625, y_half=n * 0.0625, nz=1)
    o = O.Oracle(g, cfg["phys"])
    st = o.initial(cfg["beam"])
    t0 = time.perf_counter()
    o.run(cfg["beam"], np.ones((1, n, n)), state=st)
    dt = time.perf_counter() - t0
    cells = g["nx"] * g["ny"] * g["nth"] ** 2 * g["ng"] * g["ngen"]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"1 depth step of the workload on a {n}x{n} lateral window (same cells, angles, groups, "
                      f"{g['ngen']} generations): {dt:.2f} s"}


def batched(nbeams, phys_override=None):
    """Config 4 beams (uneven energies, groups and depths; 32x32 windows of a shared phantom):
    one graph launch per wave vs the same beams run one at a time through the single-beam path."""
    import torch

    from paper_2504_00340_amd import inputs as I
    from paper_2504_00340_amd.pbsplit import Batch, Solver

    cfg = I.config4(seed=0, nbeams=nbeams)
    beams, ph = cfg["beams"], cfg["phys"]
    cells = sum(b["grid"]["nx"] * b["grid"]["ny"] * b["grid"]["nth"] ** 2 * b["grid"]["ng"] * b["grid"]["ngen"]
                * b["grid"]["nz"] for b in beams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in beams:
        s = Solver(b["grid"], ph, precision="fp32")
        s.set_phantom(b["rho"])
        s.set_beam(b["beam"])
        s.run()
        s.dose()
        s.close()
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    bt = Batch(beams, ph, wave=64)
    t0 = time.perf_counter()
    bt.run()                    # first run: includes the autotuner
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    bt.run()
    t_batch = time.perf_counter() - t0
    tuning = bt.tuning()
    bt.close()
    return {"workload": f"{cfg['name']}: first {nbeams} beams, E in "
                        f"[{min(b['beam']['e0'] for b in beams):.0f}, {max(b['beam']['e0'] for b in beams):.0f}] MeV, "
                        f"G {min(b['grid']['ng'] for b in beams)}-{max(b['grid']['ng'] for b in beams)}, "
                        f"{min(b['grid']['nz'] for b in beams)}-{max(b['grid']['nz'] for b in beams)} steps",
            "beams": nbeams, "beams_per_s": nbeams / t_batch, "beams_per_s_single_beam_path": nbeams / t_single,
            "speedup": t_single / t_batch, "cell_updates_per_s": cells / t_batch,
            "first_run_s_with_autotune": t_first, "tuning": tuning}


def surrogate(nseeds, tol=1e-2):
    """Config-5 held-out beams: the plain K = 1 march against the surrogate of generation 1 (trained
    weights shipped with the package; residual test with fallback to the plain march)."""
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
    return {"workload": f"config 5 held-out seeds 100000-{100_000 + nseeds - 1}: 64x64 cells, 16x16 angles, "
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
    ap.add_argument("--case", default="water", choices=["water", "bone", "lung"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--source", default="bf16x1", choices=["bf16x1", "bf16x2", "bf16x3", "fp32"],
                    help="arithmetic of the angular source product (FP32 contexts)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-beams", type=int, default=8,
                    help="config-4 beams for the batched leg (0 = skip)")
    ap.add_argument("--surrogate-beams", type=int, default=4,
                    help="config-5 held-out beams for the surrogate leg (0 = skip)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate leg (for profiling it alone; prints that leg's JSON object)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (scale reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU sharding is a design note, "
              "not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2504_00340_amd import inputs as I
    from paper_2504_00340_amd.pbsplit import Solver

    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate(max(1, args.surrogate_beams))}))
        return
    cfg = I.config2(args.case)
    g = cfg["grid"]
    if args.warmup + args.steps > g["nz"]:
        sys.exit(f"warmup + steps must be <= {g['nz']} depth steps")
    print(f"bench: {cfg['name']} {args.precision}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
          flush=True)
    s = Solver(g, cfg["phys"], precision=args.precision, device="cuda:0")
    split = args.precision == "fp32" and args.source != "fp32"
    nprod = {"bf16x3": 3, "bf16x2": 2, "bf16x1": 1}.get(args.source, 2)
    if args.precision == "fp32":
        from paper_2504_00340_amd.pbsplit import PBS_SRC_BF16X1, PBS_SRC_BF16X2, PBS_SRC_BF16X3, PBS_SRC_FP32

        s.set_source_precision({"bf16x1": PBS_SRC_BF16X1, "bf16x2": PBS_SRC_BF16X2,
                                "bf16x3": PBS_SRC_BF16X3}.get(args.source, PBS_SRC_FP32))
    s.set_phantom(cfg["rho"])
    s.set_beam(cfg["beam"])
    s.step(args.warmup)
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    dt = (t1 - t0) / args.steps
    cells = g["nx"] * g["ny"] * g["nth"] ** 2 * g["ng"] * g["ngen"]
    interior = g["nx"] * g["ny"] * (g["nth"] - 1) ** 2 * g["ng"] * g["ngen"]
    print("bench: kernel totals over the timed region (ms, launches): "
          + ", ".join(f"{k} {v[0]:.1f}/{v[1]}" for k, v in prof.items()), file=sys.stderr, flush=True)

    tsz = 8 if args.precision == "fp64" else 4
    alg = algorithmic(g, tsz)
    dom = max((k for k in prof if k in alg), key=lambda k: prof[k][0])
    ms, n = prof[dom]
    avg_s = ms / max(n, 1) / 1e3
    if alg[dom][0] == "bytes":
        achieved = alg[dom][1] / avg_s / 1e9
        split_ok = args.precision == "fp32" and args.case == "water" and args.source == "bf16x1"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom) if split_ok else None, "kernel": dom,
                "algorithmic_bytes_per_launch": alg[dom][1], "avg_launch_ms": avg_s * 1e3}
    else:
        mfma = args.precision == "fp32" and (g["nth"] - 1) ** 2 >= 128
        if split:
            # executed BF16 MFMA work: two or three bf16 products per FP32 multiply-add
            achieved = nprod * alg[dom][1] / avg_s / 1e12
            peak = BF16_MFMA_TFLOPS
        else:
            achieved = alg[dom][1] / avg_s / 1e12
            peak = FP32_MFMA_TFLOPS if mfma else FP32_VALU_TFLOPS
        roof = {"bound": "mfma" if mfma else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "dtype": args.source if split else args.precision,
                "traffic": measured_traffic(dom) if args.source == "bf16x1" and args.case == "water" else None,
                "kernel": dom, "algorithmic_flops_per_launch": alg[dom][1],
                "avg_launch_ms": avg_s * 1e3}
    out = {
        "metric": "phase-space cell-updates/s per z-step",
        "value": cells / dt,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: 64x64 lateral x 32x32 angles x 128 groups x 4 generations, "
                               f"300 depth steps", "steps_per_beam": g["nz"], "precision": args.precision,
                   "source_product": args.source if split else args.precision},
        "interior_cell_updates_per_s": interior / dt,
        "beams_per_s": 1.0 / (dt * g["nz"]),
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "roofline": roof,
    }
    s.close()
    if args.calibrate_copy:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n}
        del src, dst
    if args.batched_beams > 0:
        print(f"bench: batched leg, {args.batched_beams} config-4 beams", file=sys.stderr, flush=True)
        out["batched"] = batched(args.batched_beams)
    if args.surrogate_beams > 0:
        print(f"bench: surrogate leg, {args.surrogate_beams} config-5 beams", file=sys.stderr, flush=True)
        out["surrogate"] = surrogate(args.surrogate_beams)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
