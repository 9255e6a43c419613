"""Train the surrogate of generation 1 on the solver's own output, on one GPU.

  python -m paper_2504_00340_amd.train_surrogate --out <blob>      (240 beams, 30000 Adam steps)
  python -m paper_2504_00340_amd.train_surrogate --evaluate <blob> --eval-seeds 100

1. Data: for every training seed, a K = 1 beam of the surrogate workload (64 x 64 cells on
   +-4 cm, 16 x 16 angular nodes on +-0.15 rad, 96 groups on [0, E0 + 10] MeV, 300 depth steps over
   min(30, 1.25 R(E0)) cm, E0 ~ U[70, 230] MeV, seeded random layered phantom with an insert and
   +-5 % noise) is marched by the plain method in recording mode; the library writes the per-slice
   features and targets straight into device tensors.
2. Training: Adam on random minibatches of slices through pbs_net_train_step (the library's BF16
   MFMA forward/backward kernels); the learning rate decays by cosine to 5 % of its start.
3. Leak model: the fraction of the injected energy that generation 1 does not deposit, measured on
   every training beam, is fitted by least squares as l0 + l1 x + l2 x^2 in the fraction x of the
   beam energy that the primaries do not deposit; the coefficients go into the weights header,
   where the surrogate's residual test reads them.
4. Evaluation on held-out seeds: plain K = 1 dose, primaries-only dose (the method without
   generation 1), the network's dose with the residual test switched off, and the surrogate with
   its residual test and fallback; relative L2 errors against the plain K = 1 dose, residuals and
   the wall time per beam.
Every step of the solver and of the network runs in libpbsplit; torch provides device memory,
random minibatch gathers and the stream.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs as I
from .pbsplit import Net, Solver, pack_weights, param_count

H = W = 64
LAYERS = [(8, 32), (32, 32), (32, 32), (32, 1)]
TRAIN_SEED0, EVAL_SEED0 = 0, 100_000


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases; the output layer starts 10x smaller."""
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i, (ci, co) in enumerate(LAYERS):
        w = r.normal(size=(co, ci, 3, 3)) * math.sqrt(2.0 / (9 * ci))
        if i == len(LAYERS) - 1:
            w *= 0.1
        out += [w.reshape(-1), np.zeros(co)]
    p = np.concatenate(out).astype(np.float32)
    assert p.size == param_count()
    return p


def generate(seeds, nz: int = 300, log=print):
    """Features [N, 64, 64, 8] (bfloat16) and targets [N, 64, 64] (float32) of every slice of every
    seed, on the device, and per beam (seed, E0, primary escape fraction, injected energy,
    generation-1 deposit, leak fraction, primary deposit)."""
    import torch

    n = len(seeds) * nz
    X = torch.empty((n, H, W, 8), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((n, H, W), dtype=torch.float32, device="cuda")
    energy = []
    t0 = time.time()
    for k, seed in enumerate(seeds):
        c = I.config5(seed, nz)
        s = Solver(c["grid"], c["phys"], "fp32", surrogate="record")
        s.set_phantom(c["rho"])
        s.set_beam(c["beam"])
        s.run()
        s.surrogate_sample(X[k * nz:(k + 1) * nz], T[k * nz:(k + 1) * nz])
        rep = s.surrogate_report()
        energy.append((seed, c["beam"]["e0"], rep["primary_escape"], rep["injected"], rep["own_deposit"],
                       rep["leak"], rep["primary_deposit"]))
        s.close()
        if (k + 1) % 10 == 0 or k + 1 == len(seeds):
            log(f"generated {k + 1}/{len(seeds)} beams, {time.time() - t0:.1f} s", flush=True)
    return X, T, np.array(energy)


def train(X, T, steps: int, batch: int, lr: float, seed: int, log=print, weights=None):
    """Adam on random minibatches (slices drawn uniformly, or with probability proportional to `weights`,
    one per slice); returns (params, per-step losses)."""
    import torch

    n = X.shape[0]
    net = Net(H, W, batch)
    net.set_params(init_params(seed))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    wt = None if weights is None else torch.as_tensor(weights, dtype=torch.float32, device="cuda")
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda")
    t0 = time.time()
    for k in range(steps):
        if wt is None:
            idx = torch.randint(0, n, (batch,), device="cuda", generator=g)
        else:
            idx = torch.multinomial(wt, batch, replacement=True, generator=g)
        xb = X.index_select(0, idx).contiguous()
        tb = T.index_select(0, idx).contiguous()
        lr_k = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * k / steps)))
        net.train_step(xb, tb, lr_k, losses[k:k + 1])
        if (k + 1) % 1000 == 0 or k + 1 == steps:
            l = losses[max(0, k - 99):k + 1].mean().item()
            log(f"step {k + 1}/{steps} loss {l:.3e} ({time.time() - t0:.1f} s)", flush=True)
    return net.params(), losses.cpu().numpy()


def fit_leak(energy):
    """Least-squares l0 + l1 x + l2 x^2 of the measured leak fraction in the primary escape
    fraction x."""
    x, lk = energy[:, 2], energy[:, 5]
    A = np.stack([np.ones_like(x), x, x * x], axis=1)
    coef, *_ = np.linalg.lstsq(A, lk, rcond=None)
    return coef, float(np.sqrt(np.mean((A @ coef - lk) ** 2)))


def evaluate(blob: bytes, seeds, nz: int = 300, tol: float = 1e-2, log=print):
    """Per held-out seed: errors of the surrogate (with and without its residual test) and of the
    primaries-only march against the plain K = 1 march, the residual, fallback flag and wall times
    (ms per beam)."""
    import torch

    rows = []
    for seed in seeds:
        c = I.config5(seed, nz)
        out = {}
        for mode in ("plain", "primaries", "net", "surrogate"):
            g = dict(c["grid"], ngen=1) if mode == "primaries" else c["grid"]
            sur = blob if mode in ("net", "surrogate") else None
            s = Solver(g, c["phys"], "fp32", surrogate=sur, residual_tol=1e30 if mode == "net" else tol)
            s.set_phantom(c["rho"])
            best = None
            for rep in range(2):            # the first run warms up
                s.set_beam(c["beam"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.run()
                r = s.surrogate_report() if sur else None   # synchronises
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            out[mode] = (s.dose(), best * 1e3, r)
            s.close()
        ref = out["plain"][0]
        nrm = np.linalg.norm(ref)
        row = dict(seed=seed, e0=c["beam"]["e0"],
                   err_net=float(np.linalg.norm(out["net"][0] - ref) / nrm),
                   err_surrogate=float(np.linalg.norm(out["surrogate"][0] - ref) / nrm),
                   err_primaries=float(np.linalg.norm(out["primaries"][0] - ref) / nrm),
                   residual=out["surrogate"][2]["residual"], fallback=out["surrogate"][2]["fallback"],
                   leak_model=out["surrogate"][2]["leak"], ms_plain=out["plain"][1],
                   ms_primaries=out["primaries"][1], ms_net=out["net"][1], ms_surrogate=out["surrogate"][1])
        rows.append(row)
        log(json.dumps(row), flush=True)
    return rows


def summarize(rows):
    """Accept rate, error distribution of the accepted beams and of the network alone, throughput."""
    acc = [r for r in rows if not r["fallback"]]
    en = np.array([r["err_net"] for r in rows])
    ea = np.array([r["err_surrogate"] for r in acc]) if acc else np.zeros(0)
    out = dict(accepted=len(acc), accept_rate=len(acc) / len(rows),
               mean_err_net=float(en.mean()), max_err_net=float(en.max()),
               p90_err_net=float(np.percentile(en, 90)),
               mean_err_surrogate=float(np.mean([r["err_surrogate"] for r in rows])),
               max_err_surrogate=float(np.max([r["err_surrogate"] for r in rows])),
               mean_err_accepted=float(ea.mean()) if acc else None, max_err_accepted=float(ea.max()) if acc else None,
               mean_err_primaries=float(np.mean([r["err_primaries"] for r in rows])),
               fallback_energies=[r["e0"] for r in rows if r["fallback"]],
               beams_per_s_plain=len(rows) / (np.sum([r["ms_plain"] for r in rows]) * 1e-3),
               beams_per_s_surrogate=len(rows) / (np.sum([r["ms_surrogate"] for r in rows]) * 1e-3),
               speedup=float(np.sum([r["ms_plain"] for r in rows]) / np.sum([r["ms_surrogate"] for r in rows])))
    for lo, hi in ((70, 130), (130, 190), (190, 230)):
        sel = [r for r in rows if lo <= r["e0"] < hi]
        if sel:
            out[f"band_{lo}_{hi}"] = dict(n=len(sel), accepted=sum(1 for r in sel if not r["fallback"]),
                                          mean_err_net=float(np.mean([r["err_net"] for r in sel])),
                                          max_err_net=float(np.max([r["err_net"] for r in sel])))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-seeds", type=int, default=240)
    ap.add_argument("--eval-seeds", type=int, default=8)
    ap.add_argument("--nz", type=int, default=300)
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--energy-weight", type=float, default=0.0, metavar="P",
                    help="draw a beam's slices with weight (E0 / 150 MeV)^P (0: uniform)")
    ap.add_argument("--out", default=None, help="weights blob to write")
    ap.add_argument("--evaluate", default=None, metavar="BLOB",
                    help="skip data and training: evaluate this weights blob on the held-out seeds")
    ap.add_argument("--report", default=None, help="JSON summary to write")
    a = ap.parse_args(argv)
    if a.evaluate:
        with open(a.evaluate, "rb") as f:
            blob = f.read()
        rows = evaluate(blob, range(EVAL_SEED0, EVAL_SEED0 + a.eval_seeds), a.nz)
        summary = dict(weights=a.evaluate, eval_seeds=a.eval_seeds, **summarize(rows), eval=rows)
        print(json.dumps({k: v for k, v in summary.items() if k != "eval"}), flush=True)
        if a.report:
            with open(a.report, "w") as f:
                json.dump(summary, f, indent=1)
        return
    if not a.out:
        ap.error("--out is required unless --evaluate is given")
    X, T, energy = generate(range(TRAIN_SEED0, TRAIN_SEED0 + a.train_seeds), a.nz)
    leak, leak_rms = fit_leak(energy)
    print(f"generation-1 leak fraction {energy[:, 5].min():.3f} .. {energy[:, 5].max():.3f}; model "
          f"{leak.tolist()} rms {leak_rms:.3e}; injected / primary deposit "
          f"{np.mean(energy[:, 3] / energy[:, 6]):.3e}", flush=True)
    weights = None
    if a.energy_weight:
        weights = np.repeat((energy[:, 1] / 150.0) ** a.energy_weight, a.nz)
    params, losses = train(X, T, a.steps, a.batch, a.lr, a.seed, weights=weights)
    del X, T
    blob = pack_weights(params, leak)
    with open(a.out, "wb") as f:
        f.write(blob)
    rows = evaluate(blob, range(EVAL_SEED0, EVAL_SEED0 + a.eval_seeds), a.nz)
    summary = dict(train_seeds=a.train_seeds, slices=a.train_seeds * a.nz, steps=a.steps, batch=a.batch, lr=a.lr,
                   energy_weight=a.energy_weight,
                   leak_model=leak.tolist(), leak_rms=leak_rms, final_loss=float(losses[-100:].mean()), eval=rows,
                   train_beams=energy.tolist(), **summarize(rows))
    print(json.dumps({k: v for k, v in summary.items() if k not in ("eval", "train_beams")}), flush=True)
    if a.report:
        with open(a.report, "w") as f:
            json.dump(summary, f, indent=1)


if __name__ == "__main__":
    main()
