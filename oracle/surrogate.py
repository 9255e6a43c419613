"""FP64 CPU reference of the surrogate of generation 1: its per-slice features and its network.

TEST INFRASTRUCTURE ONLY: the test-suite and ``__graft_entry__.smoke()`` are the only callers; the
product path never imports this module, and nothing here is shared with the HIP path.

The surrogate is not part of the paper.  It replaces the first catastrophic-scatter generation of
the scattering decomposition (section 3.1, the source iteration of generations) by a learned
estimate of the energy that generation deposits, from records of the primary march:
  I     energy the re-emission source injects into generation 1 in layer s,
  M_E   energy content of the primaries after the opening energy half-step of layer s,
  M_N   number content of the primaries at the same point,
  E0    deposit of the primaries alone,
all per lateral cell (see ``Oracle.run_records``).  The definitions below are written out plainly
(numpy, float64, no blocking).

Network: four 3x3 convolutions with zero padding (cross-correlation, as in the usual deep-learning
definition), channels 8 -> 32 -> 32 -> 32 -> 1, ReLU after the first three; loss = mean over pixels
of (y - t)^2.  Parameters are one flat vector in the order w0, b0, w1, b1, w2, b2, w3, b3 with
w_l of shape [cout][cin][3][3].
"""
from __future__ import annotations

import numpy as np

LAYERS = [(8, 32), (32, 32), (32, 32), (32, 1)]
FILTER_L = (0.5, 2.0, 6.0, 15.0)   # cm water-equivalent, depth filters of the injected energy
E_REF = 250.0                      # MeV, scale of the mean-energy channel
NFEAT = 8


def param_count() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unflatten(p):
    """Flat parameter vector -> list of (w [co, ci, 3, 3], b [co]) as float64."""
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for ci, co in LAYERS:
        w = p[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = p[o:o + co]
        o += co
        out.append((w, b))
    assert o == p.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in layers])


def conv3x3(x, w, b):
    """x [n, H, W, ci] -> [n, H, W, co]: out = b + sum_{ky,kx} x[y+ky-1, x+kx-1, :] . w[:, :, ky, kx]."""
    n, H, W, _ = x.shape
    xp = np.zeros((n, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    out = np.zeros((n, H, W, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, :, ky, kx].T
    return out


def bf16(a):
    """Round float64 values to bfloat16 (through float32, round to nearest, ties to even), returned
    as float64: keep the top 16 bits of the float32 pattern after adding 0x7FFF plus the lowest
    kept bit."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def forward(p, x, act_bf16=False):
    """y [n, H, W] and the activations [x, a1, a2, a3] (inputs of the four layers).  act_bf16:
    the hidden activations are stored as bfloat16 (the network a BF16 implementation evaluates)."""
    L = unflatten(p)
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for i, (w, b) in enumerate(L):
        z = conv3x3(h, w, b)
        if i < 3:
            h = np.maximum(z, 0.0)
            if act_bf16:
                h = bf16(h)
            acts.append(h)
        else:
            h = z
    return h[..., 0], acts


def loss_grad(p, x, t, act_bf16=False):
    """(loss, gradient with respect to the flat parameters).  With act_bf16 the forward stores
    BF16 activations and the backward passes through the rounding as the identity."""
    L = unflatten(p)
    y, acts = forward(p, x, act_bf16)
    npx = y.size
    d = y - np.asarray(t, dtype=np.float64)
    loss = float((d * d).sum() / npx)
    gz = (2.0 * d / npx)[..., None]          # d loss / d (output of layer 3)
    grads = [None] * 4
    for i in range(3, -1, -1):
        w, _ = L[i]
        a = acts[i]
        n, H, W, ci = a.shape
        ap = np.zeros((n, H + 2, W + 2, ci))
        ap[:, 1:H + 1, 1:W + 1, :] = a
        gw = np.zeros_like(w)
        ga = np.zeros((n, H + 2, W + 2, ci))
        for ky in range(3):
            for kx in range(3):
                win = ap[:, ky:ky + H, kx:kx + W, :].reshape(-1, ci)
                gw[:, :, ky, kx] = gz.reshape(-1, w.shape[0]).T @ win
                ga[:, ky:ky + H, kx:kx + W, :] += gz @ w[:, :, ky, kx]
        grads[i] = (gw, gz.sum(axis=(0, 1, 2)))
        if i > 0:
            # through the ReLU that produced this layer's input
            gz = ga[:, 1:H + 1, 1:W + 1, :] * (a > 0)
    return loss, flatten(grads)


def scale(rec):
    """Feature scale c = max of the injected energy over the beam."""
    c = float(rec[0].max())
    return c if c > 0 else 1.0


def features(rec, rho, dz, kappa0):
    """Per-slice features [nz, nx, ny, 8] from the records and the densities [nz, nx, ny]:
    M_E kappa0 dz / c, rho, I / c, F_0.5 / c, F_2 / c, F_6 / c, mean primary energy / 250 MeV,
    F_15 / c."""
    I, ME, MN = rec[0], rec[1], rec[2]
    c = scale(rec)
    cn = float(MN.max())
    nz = I.shape[0]
    F = np.zeros((4,) + I.shape)
    run = np.zeros((4,) + I.shape[1:])
    for s in range(nz):
        for j, Lj in enumerate(FILTER_L):
            a = np.exp(-rho[s] * dz / Lj)
            run[j] = a * run[j] + (1.0 - a) * I[s]
            F[j, s] = run[j]
    eb = np.where(MN > 1e-4 * cn, ME / np.where(MN > 1e-4 * cn, MN, 1.0), 0.0) if cn > 0 else np.zeros_like(ME)
    X = np.stack([ME * kappa0 * dz / c, rho, I / c, F[0] / c, F[1] / c, F[2] / c, eb / E_REF, F[3] / c], axis=-1)
    return X


def target(rec, edep_total):
    """Energy generation 1 deposits itself per voxel, over c: (E_total - E0 + I) / c."""
    return (edep_total - rec[3] + rec[0]) / scale(rec)


def surrogate_edep(rec, y):
    """Deposit of the surrogate march: E0 - I + c * y."""
    return rec[3] - rec[0] + scale(rec) * y
