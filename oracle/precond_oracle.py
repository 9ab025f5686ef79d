"""ORACLE -- test infrastructure, not part of the product.

Plain FP64 numpy reference of the learned correction to the block-Jacobi
preconditioner of the reduced camera system.  Only the test suite may
import this module; the GPU library shares no code with it.

The paper preconditions its PCG with a diagonal (block) preconditioner
(Sec. IV-C-2).  The learned variant keeps that structure and corrects each
9x9 block from the camera co-visibility graph:

  S_ii = L_i L_i^T (Cholesky), S^_ij = L_i^-1 S_ij L_j^-T (normalised
  coupling; the normalised diagonal blocks are I), E_i = sum_{j != i}
  S^_ij S^_ij^T, a_ij = |S^_ij|_F.

  node input x_i = [upper(E_i) (45), log(1 + tr E_i), log(1 + deg_i)]
  h0_i = relu(W_in x_i + b_in)
  for l = 1..3:  m_i = sum_j a_ij h_j / sum_j a_ij   (0 without neighbours)
                 h_i = relu(W_s h_i + W_m m_i + b)
  o_i = W_out h_i + b_out (45 = lower triangle of a 9x9, row-major)
  C_i = strict lower part of o_i + diag(exp(o_i,diag))
  M_i = L_i^-T C_i C_i^T L_i^-1      (SPD; o = 0 gives block-Jacobi exactly)

Training loss of one system: the squared Frobenius distance of the
normalised preconditioned operator to the identity, which decomposes over
the block rows because M is block diagonal:
  loss = (1/n) sum_i tr(Mh_i G_i Mh_i) - 2 tr(Mh_i) + 9,
  Mh_i = C_i C_i^T, G_i = I + E_i,
minimised by Mh_i = G_i^-1.
"""
from __future__ import annotations

import numpy as np

HID = 64
NF = 47
NOUT = 45
LAYERS = 3

_UPPER = [(r, c) for r in range(9) for c in range(r, 9)]
_LOWER = [(r, c) for r in range(9) for c in range(r + 1)]


def param_shapes():
    shapes = [("W_in", (HID, NF)), ("b_in", (HID,))]
    for l in range(LAYERS):
        shapes += [(f"W_s{l}", (HID, HID)), (f"W_m{l}", (HID, HID)), (f"b{l}", (HID,))]
    shapes += [("W_out", (NOUT, HID)), ("b_out", (NOUT,))]
    return shapes


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def unpack(theta):
    out, k = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        out[name] = theta[k:k + n].reshape(shp)
        k += n
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in param_shapes()])


def init_params(rng) -> np.ndarray:
    """He-scaled hidden layers, zero output layer (starts at block-Jacobi)."""
    d = {}
    for name, shp in param_shapes():
        if name.startswith("W") and name != "W_out":
            d[name] = rng.normal(size=shp) * np.sqrt(2.0 / shp[1])
        else:
            d[name] = np.zeros(shp)
    return pack(d)


def system_graph(S_ptr, S_col, S_blocks, nc):
    """Graph of one reduced camera system given as its upper block pattern
    (rows S_ptr/S_col, blocks [nnzb, 9, 9], diagonal included)."""
    diag = np.zeros((nc, 9, 9))
    offd = []
    for a in range(nc):
        for e in range(S_ptr[a], S_ptr[a + 1]):
            b = int(S_col[e])
            if b == a:
                diag[a] = S_blocks[e]
            else:
                offd.append((a, b, S_blocks[e]))
    L = np.linalg.cholesky(diag)
    Linv = np.linalg.inv(L)
    E = np.zeros((nc, 9, 9))
    nbr = [[] for _ in range(nc)]
    for a, b, B in offd:
        Sh = Linv[a] @ B @ Linv[b].T
        E[a] += Sh @ Sh.T
        E[b] += Sh.T @ Sh
        w = np.linalg.norm(Sh)
        nbr[a].append((b, w))
        nbr[b].append((a, w))
    X = np.zeros((nc, NF))
    for i in range(nc):
        X[i, :45] = [E[i][r, c] for r, c in _UPPER]
        X[i, 45] = np.log1p(np.trace(E[i]))
        X[i, 46] = np.log1p(len(nbr[i]))
    # aggregation matrix P: m = P h, P_ij = a_ij / sum_j a_ij
    P = np.zeros((nc, nc))
    for i in range(nc):
        tot = sum(w for _, w in nbr[i])
        for j, w in nbr[i]:
            if tot > 0:
                P[i, j] += w / tot
    return {"nc": nc, "L": L, "Linv": Linv, "E": E, "X": X, "P": P, "diag": diag}


def bf16(a):
    """Rounding to bfloat16 (8 significant bits) by its definition: the value
    as float32, the low 16 bits of its encoding dropped with round-to-nearest,
    ties to even; returned as float64."""
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, g, bf16_inference=False):
    """Node outputs o and the activations.  bf16_inference: the message
    layers take their operands (inputs, weights) rounded to bfloat16, as the
    matrix-core inference does (its input layer stays unrounded); sums and
    biases stay exact here."""
    p = unpack(theta)
    X, P = g["X"], g["P"]
    q = bf16 if bf16_inference else (lambda v: v)
    z0 = X @ p["W_in"].T + p["b_in"]
    h = np.maximum(z0, 0.0)
    cache = {"z": [z0], "h": [h], "m": []}
    for l in range(LAYERS):
        m = P @ h
        z = q(h) @ q(p[f"W_s{l}"]).T + q(m) @ q(p[f"W_m{l}"]).T + p[f"b{l}"]
        h = np.maximum(z, 0.0)
        cache["m"].append(m)
        cache["z"].append(z)
        cache["h"].append(h)
    o = h @ p["W_out"].T + p["b_out"]
    return o, cache


def C_from_o(o):
    n = o.shape[0]
    C = np.zeros((n, 9, 9))
    for t, (r, c) in enumerate(_LOWER):
        C[:, r, c] = np.exp(o[:, t]) if r == c else o[:, t]
    return C


def loss_from_C(C, g):
    n = g["nc"]
    Mh = C @ np.transpose(C, (0, 2, 1))
    G = np.eye(9) + g["E"]
    val = np.einsum("nij,njk,nki->", Mh, G, Mh) - 2.0 * np.einsum("nii->", Mh) + 9.0 * n
    return val / n


def dloss_dC(C, g):
    n = g["nc"]
    Mh = C @ np.transpose(C, (0, 2, 1))
    G = np.eye(9) + g["E"]
    Gam = (G @ Mh + Mh @ G - 2.0 * np.eye(9)) / n       # d loss / d Mh (symmetric)
    return 2.0 * Gam @ C


def loss(theta, g):
    o, _ = forward(theta, g)
    return loss_from_C(C_from_o(o), g)


def grad(theta, g):
    """d loss / d theta by reverse-mode differentiation written out."""
    p = unpack(theta)
    o, cache = forward(theta, g)
    C = C_from_o(o)
    dC = dloss_dC(C, g)
    do = np.zeros_like(o)
    for t, (r, c) in enumerate(_LOWER):
        do[:, t] = dC[:, r, c] * (C[:, r, c] if r == c else 1.0)
    gr = {}
    h = cache["h"][-1]
    gr["W_out"] = do.T @ h
    gr["b_out"] = do.sum(0)
    dh = do @ p["W_out"]
    for l in reversed(range(LAYERS)):
        dz = dh * (cache["z"][l + 1] > 0)
        hp, m = cache["h"][l], cache["m"][l]
        gr[f"W_s{l}"] = dz.T @ hp
        gr[f"W_m{l}"] = dz.T @ m
        gr[f"b{l}"] = dz.sum(0)
        dm = dz @ p[f"W_m{l}"]
        dh = dz @ p[f"W_s{l}"] + g["P"].T @ dm
    dz0 = dh * (cache["z"][0] > 0)
    gr["W_in"] = dz0.T @ g["X"]
    gr["b_in"] = dz0.sum(0)
    return pack(gr)


def precond_blocks(theta, g, bf16_inference=False):
    """M_i = L_i^-T C_i C_i^T L_i^-1 for every camera."""
    o, _ = forward(theta, g, bf16_inference)
    C = C_from_o(o)
    Li = g["Linv"]
    return np.transpose(Li, (0, 2, 1)) @ C @ np.transpose(C, (0, 2, 1)) @ Li


def pcg_iterations(S_ptr, S_col, S_blocks, b, Mblocks, rtol, maxiter):
    """Textbook PCG (x0 = 0) on the symmetric system given by its upper
    blocks, preconditioned by the block-diagonal M; returns the iteration
    count at which |b - S x| <= rtol |b| (recursive residual)."""
    nc = len(S_ptr) - 1

    def spmv(x):
        X = x.reshape(nc, 9)
        Y = np.zeros_like(X)
        for a in range(nc):
            for e in range(S_ptr[a], S_ptr[a + 1]):
                c = int(S_col[e])
                Y[a] += S_blocks[e] @ X[c]
                if c != a:
                    Y[c] += S_blocks[e].T @ X[a]
        return Y.reshape(-1)

    def prec(r):
        return np.einsum("nij,nj->ni", Mblocks, r.reshape(nc, 9)).reshape(-1)

    b = np.asarray(b, np.float64).reshape(-1)
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r)
    pdir = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    for k in range(1, maxiter + 1):
        q = spmv(pdir)
        alpha = rz / (pdir @ q)
        x += alpha * pdir
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            return k
        z = prec(r)
        rz2 = r @ z
        pdir = z + (rz2 / rz) * pdir
        rz = rz2
    return maxiter
