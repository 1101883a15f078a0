"""FP64 NumPy reference of the learned surrogate (forward, loss, backward).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper has no
learned component; this file is the definition the GPU's BF16-MFMA kernels
are checked against.  It shares no code with the GPU library.

Network (tokens = patches of 4 nodes of one tube):
  X  [M,16]   feature p*4+c of token t = (v_c(node 4t+p) - mu_c) / sd_c,
              v = (rho, u, T, gamma), mu = (0.5, 0, 1, 1.4), sd = (0.5, 0.5, 0.5, 0.3)
  H0 = X We^T + be
  block: Hc = H + bc + sum_k kc[:,k] * H[t+k-2]   (per channel; zero outside
         the tube's tokens), H' = Hc + W2 gelu(W1 Hc + b1) + b2
  Y  = H4 Wh^T + bh,  y_c(node 4t+p) = x_c + 0.1 Y[t, 3p+c]
  loss = mean over tokens and the 12 outputs of (Y - (target - x)/0.1)^2
Parameter vector: We[64,16], be[64], 4 x {kc[64,5], bc[64], W1[128,64],
b1[128], W2[64,128], b2[64]}, Wh[12,64], bh[12]  (69708 values).

rounded=True applies round-to-nearest-even BF16 at the points where the GPU
rounds (matrix-product operands, the input features, the GELU output and the
back-propagated matrix-product inputs); rounded=False is a plain FP64 network.
"""
from __future__ import annotations

import numpy as np

C, HID, NB, TAPS, FIN, FOUT, PATCH = 64, 128, 4, 5, 16, 12, 4
MU = np.array([0.5, 0.0, 1.0, 1.4])
SD = np.array([0.5, 0.5, 0.5, 0.3])
OUT_SCALE = 0.1


def layout():
    """[(name, shape)] in parameter-vector order."""
    items = [("We", (C, FIN)), ("be", (C,))]
    for b in range(NB):
        items += [(f"kc{b}", (C, TAPS)), (f"bc{b}", (C,)), (f"W1{b}", (HID, C)), (f"b1{b}", (HID,)),
                  (f"W2{b}", (C, HID)), (f"b2{b}", (C,))]
    items += [("Wh", (FOUT, C)), ("bh", (FOUT,))]
    return items


NPARAMS = sum(int(np.prod(s)) for _, s in layout())


def unpack(vec):
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in layout()])


def bf16(a):
    """Round to the nearest BF16 (ties to even), via FP32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _gelu(z):
    k = np.sqrt(2.0 / np.pi)
    return 0.5 * z * (1.0 + np.tanh(k * (z + 0.044715 * z ** 3)))


def _gelu_grad(z):
    k = np.sqrt(2.0 / np.pi)
    t = np.tanh(k * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * k * (1.0 + 3.0 * 0.044715 * z * z)


def tokens(x, gamma):
    """x [3,B,L] (rho,u,T), gamma [B] -> X [M,16] (unrounded)."""
    _, B, L = x.shape
    T = L // PATCH
    v = np.concatenate([x, np.broadcast_to(gamma[None, :, None], (1, B, L))], axis=0)  # [4,B,L]
    v = (v - MU[:, None, None]) / SD[:, None, None]
    v = v.reshape(4, B, T, PATCH).transpose(1, 2, 3, 0)  # [B,T,p,c]
    return v.reshape(B * T, FIN)


def _conv(H, kc, T):
    """sum_k kc[c,k] H[t+k-2, c] within each tube (zero padding)."""
    M = H.shape[0]
    Hb = H.reshape(M // T, T, C)
    out = np.zeros_like(Hb)
    for k in range(TAPS):
        s = k - 2
        if s >= 0:
            out[:, :T - s] += kc[None, None, :, k] * Hb[:, s:]
        else:
            out[:, -s:] += kc[None, None, :, k] * Hb[:, :T + s]
    return out.reshape(M, C)


def _conv_t(D, kc, T):
    """Adjoint of _conv: out[t] = sum_k kc[c,k] D[t-k+2]."""
    M = D.shape[0]
    Db = D.reshape(M // T, T, C)
    out = np.zeros_like(Db)
    for k in range(TAPS):
        s = k - 2  # D[t] feeds out[t+s]
        if s >= 0:
            out[:, s:] += kc[None, None, :, k] * Db[:, :T - s]
        else:
            out[:, :T + s] += kc[None, None, :, k] * Db[:, -s:]
    return out.reshape(M, C)


def forward(p, x, gamma, rounded=True):
    r = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    _, B, L = x.shape
    T = L // PATCH
    X = r(tokens(x, gamma))
    act = {"X": X, "T": T}
    H = X @ r(p["We"]).T + p["be"]
    act["H0"] = H
    for b in range(NB):
        Hc = H + p[f"bc{b}"] + _conv(H, p[f"kc{b}"], T)
        Z1 = r(Hc) @ r(p[f"W1{b}"]).T + p[f"b1{b}"]
        A1 = r(_gelu(Z1))
        H = Hc + A1 @ r(p[f"W2{b}"]).T + p[f"b2{b}"]
        act[f"Hc{b}"], act[f"Z1{b}"], act[f"A1{b}"], act[f"H{b + 1}"] = Hc, Z1, A1, H
    Y = r(H) @ r(p["Wh"]).T + p["bh"]
    act["Y"] = Y
    y = x + OUT_SCALE * Y.reshape(B, T, PATCH, 3).transpose(3, 0, 1, 2).reshape(3, B, L)
    return y, act


def loss_and_grads(p, x, gamma, target, rounded=True):
    """(loss, grads dict, y) for loss = mean((Y - (target - x)/0.1)^2)."""
    r = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    _, B, L = x.shape
    T = L // PATCH
    y, a = forward(p, x, gamma, rounded)
    M = B * T
    tn = ((target - x) / OUT_SCALE).reshape(3, B, T, PATCH).transpose(1, 2, 3, 0).reshape(M, FOUT)
    diff = a["Y"] - tn
    loss = float(np.mean(diff ** 2))
    dY = r(2.0 * diff / (M * FOUT))
    g = {}
    H4 = a[f"H{NB}"]
    g["Wh"] = dY.T @ r(H4)
    g["bh"] = dY.sum(0)
    dH = dY @ r(p["Wh"])
    for b in reversed(range(NB)):
        dO = dH
        dA1 = r(dO) @ r(p[f"W2{b}"])
        dZ1 = r(dA1 * _gelu_grad(a[f"Z1{b}"]))
        g[f"W2{b}"] = r(dO).T @ a[f"A1{b}"]
        g[f"b2{b}"] = r(dO).sum(0)
        g[f"W1{b}"] = dZ1.T @ r(a[f"Hc{b}"])
        g[f"b1{b}"] = dZ1.sum(0)
        dHc = dO + dZ1 @ r(p[f"W1{b}"])
        Hin = a[f"H{b}"] if b > 0 else a["H0"]
        Hb = Hin.reshape(B, T, C)
        Db = dHc.reshape(B, T, C)
        gk = np.zeros((C, TAPS))
        for k in range(TAPS):
            s = k - 2
            if s >= 0:
                gk[:, k] = (Db[:, :T - s] * Hb[:, s:]).sum((0, 1))
            else:
                gk[:, k] = (Db[:, -s:] * Hb[:, :T + s]).sum((0, 1))
        g[f"kc{b}"] = gk
        g[f"bc{b}"] = dHc.sum(0)
        dH = dHc + _conv_t(dHc, p[f"kc{b}"], T)
    g["We"] = r(dH).T @ a["X"]
    g["be"] = r(dH).sum(0)
    return loss, g, y


def init_params(seed=0):
    """Seeded initial parameters (the GPU trainer uses the same recipe)."""
    rng = np.random.default_rng(seed)
    d = {"We": rng.normal(0, 1 / np.sqrt(FIN), (C, FIN)), "be": np.zeros(C)}
    for b in range(NB):
        d[f"kc{b}"] = rng.normal(0, 0.1, (C, TAPS))
        d[f"bc{b}"] = np.zeros(C)
        d[f"W1{b}"] = rng.normal(0, 1 / np.sqrt(C), (HID, C))
        d[f"b1{b}"] = np.zeros(HID)
        d[f"W2{b}"] = rng.normal(0, 0.2 / np.sqrt(HID), (C, HID))
        d[f"b2{b}"] = np.zeros(C)
    d["Wh"] = rng.normal(0, 0.01, (FOUT, C))
    d["bh"] = np.zeros(FOUT)
    return pack(d)


def adam(p, m, v, g, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return p, m, v
