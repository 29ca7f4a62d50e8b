"""CPU oracle of the learned R surrogate: features, MLP, gradients, Adam.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`).  Plain numpy in FP64,
written from the definitions below; the GPU library shares no code with it.

The paper computes R exactly from nearest neighbours (Sec. 2.2, the local
velocity density and the ratio to the background Gaussian).  The surrogate
predicts that R from cheap per-particle inputs and is judged against the
exact value; everything here is therefore a plain definition:

Features (12 per particle k of a searched host, Sigma(x_k) with eigenvalues
lam_1 <= lam_2 <= lam_3 and unit eigenvectors e_a, dv = v_k - vbar(x_k)):
  0      ln rhat, rhat = (3 n_se / (4 pi nhat))^(1/3): the radius that would
         hold n_se neighbours at the count density nhat of the 27 fine cells
         around the particle (cell side f = 2^cell_bits grid units), or of the
         27 coarse cells (side 4 f) when the fine window holds fewer than n_se
         host members;
  1..3   |dv . e_a| / sqrt(lam_a);
  4..6   ln lam_a;
  7      ln rho_cell (density of the particle's KD cell);
  8..10  |(vloc - vbar) . e_a| / sqrt(lam_a), vloc = the mean velocity of the
         host members in the particle's fine cell and its six face neighbours;
  11     |v_k - vloc| / sigma_iso, sigma_iso = sqrt((lam_1+lam_2+lam_3)/3).
Cells are counted over the members of all searched hosts together.  Absolute
values drop the arbitrary orientation of each eigenvector.  A particle whose
Sigma is not positive definite gets NaN features (the exact path decides it).

MLP 12 -> 64 -> 64 -> 64 -> 1 with ReLU.  Parameters in one FP32 vector of
MLP_PARAMS values: W1[12][64], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
w4[64], b4 (W[i][o]: input i, output o).  The inference arithmetic is BF16
inputs, weights and hidden activations with wide accumulation; the last layer
takes the FP32 activations of layer 3.  Loss = mean of (Rhat - R)^2.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 12
HID = 64
MLP_PARAMS = 12 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1  # 9217


# ---- BF16 rounding ----------------------------------------------------------
def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), via FP32.  BF16 keeps
    the top 16 bits of the FP32 pattern; NaN stays NaN."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out).reshape(np.shape(x))


def bf16_bits(x):
    """The uint16 patterns of bf16_round(x)."""
    r = bf16_round(x).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16)


def bf16_from_bits(b):
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


# ---- parameters --------------------------------------------------------------
def unpack(w):
    w = np.asarray(w, np.float64)
    assert w.shape == (MLP_PARAMS,)
    o = 0
    out = []
    for shape in ((12, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)):
        size = int(np.prod(shape))
        out.append(w[o:o + size].reshape(shape))
        o += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


# ---- forward / backward -------------------------------------------------------
def forward(w, X, bf16=True):
    """Rhat for rows X (m x 12).  bf16=True applies the inference rounding
    (inputs, W1..W3 and the activations feeding layers 2 and 3 in BF16)."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(w)
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    H0 = q(X)
    H1 = np.maximum(H0 @ q(W1) + b1, 0.0)
    H2 = np.maximum(q(H1) @ q(W2) + b2, 0.0)
    H3 = np.maximum(q(H2) @ q(W3) + b3, 0.0)
    return H3 @ w4 + b4[0]


def loss_and_grad(w, X, y, bf16=False):
    """Mean squared error and its gradient, FP64.  bf16=False: the exact
    gradient of the unrounded network.  bf16=True: the arithmetic of the
    training kernels written out: the forward pass of `forward(bf16=True)`,
    and BF16 rounding of the two factors of every weight-gradient product
    (errors and activations) and of the weights and errors that carry the
    error down a layer; bias gradients, the last layer and the ReLU masks use
    the unrounded values."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(w)
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    X = q(np.asarray(X, np.float64))
    y = np.asarray(y, np.float64)
    m = X.shape[0]
    H1 = np.maximum(X @ q(W1) + b1, 0.0)
    H2 = np.maximum(q(H1) @ q(W2) + b2, 0.0)
    H3 = np.maximum(q(H2) @ q(W3) + b3, 0.0)
    out = H3 @ w4 + b4[0]
    r = out - y
    loss = np.mean(r * r)
    g = 2.0 * r / m                       # dL/dout
    gw4 = H3.T @ g
    gb4 = np.array([g.sum()])
    d3 = np.outer(g, w4) * (H3 > 0)       # dL/dZ3 (Z > 0 exactly where H > 0)
    gW3 = q(H2).T @ q(d3)
    gb3 = d3.sum(0)
    d2 = (q(d3) @ q(W3).T) * (H2 > 0)
    gW2 = q(H1).T @ q(d2)
    gb2 = d2.sum(0)
    d1 = (q(d2) @ q(W2).T) * (H1 > 0)
    gW1 = X.T @ q(d1)
    gb1 = d1.sum(0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gw4, gb4])


def adam_step(w, m1, m2, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, with bias correction) at step t >= 1."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** t)
    vh = m2 / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2


# ---- features -------------------------------------------------------------------
def _cell_table(keys):
    u, inv, cnt = np.unique(keys, return_inverse=True, return_counts=True)
    return u, inv, cnt


def _lookup(u, vals, keys):
    """vals[u == key] for each key, 0 where the cell is empty."""
    pos = np.searchsorted(u, keys)
    pos = np.minimum(pos, len(u) - 1)
    hit = u[pos] == keys
    return np.where(hit[..., None] if vals.ndim > 1 else hit, vals[pos], 0)


def _key(c, b):
    return (c[2].astype(np.int64) << (2 * b)) | (c[1].astype(np.int64) << b) | c[0].astype(np.int64)


def features(q, v, members, vbar, sigma, rho_cell, n_se, cell_bits, box, grid_bits):
    """The 12 raw features (FP64, rows in the order of `members`)."""
    members = np.asarray(members, np.int64)
    m = len(members)
    gb = grid_bits
    qm = np.asarray(q, np.int64)[:, members]
    vm = np.asarray(v, np.float64)[:, members]
    unit = box / 2.0 ** gb
    NB = np.array([[dx, dy, dz] for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    FACES = np.array([[0, 0, 0], [-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]])

    def window(c_bits, offsets, vals):
        b = gb - c_bits
        nc = 1 << b
        c = qm >> c_bits
        u, inv, cnt = _cell_table(_key(c, b))
        table = cnt.astype(np.float64) if vals is None else np.column_stack(
            [cnt.astype(np.float64)] + [np.bincount(inv, weights=vals[d], minlength=len(u)) for d in range(3)])
        acc = np.zeros(m) if vals is None else np.zeros((m, 4))
        for o in offsets:
            cc = (c + o[:, None]) % nc
            acc = acc + _lookup(u, table, _key(cc, b))
        return acc

    n_fine = window(cell_bits, NB, None)
    n_coarse = window(cell_bits + 2, NB, None)
    f = 2.0 ** cell_bits * unit
    nhat = np.where(n_fine >= n_se, n_fine / (27.0 * f ** 3), n_coarse / (27.0 * (4.0 * f) ** 3))
    rhat = (3.0 * n_se / (4.0 * np.pi * nhat)) ** (1.0 / 3.0)
    loc = window(cell_bits, FACES, vm)
    vloc = loc[:, 1:4] / loc[:, 0:1]

    vb = np.asarray(vbar, np.float64)[:, members].T
    sg = np.asarray(sigma, np.float64)[:, members].T
    S = np.empty((m, 3, 3))
    S[:, 0, 0], S[:, 1, 1], S[:, 2, 2] = sg[:, 0], sg[:, 1], sg[:, 2]
    S[:, 0, 1] = S[:, 1, 0] = sg[:, 3]
    S[:, 0, 2] = S[:, 2, 0] = sg[:, 4]
    S[:, 1, 2] = S[:, 2, 1] = sg[:, 5]
    lam, E = np.linalg.eigh(S)            # ascending eigenvalues, eigenvectors in columns
    dv = vm.T - vb
    dl = vloc - vb
    out = np.empty((m, N_FEAT))
    ok = lam[:, 0] > 0
    sl = np.sqrt(np.where(ok[:, None], lam, 1.0))
    out[:, 0] = np.log(rhat)
    out[:, 1:4] = np.abs(np.einsum("mi,mia->ma", dv, E)) / sl
    out[:, 4:7] = np.log(np.where(ok[:, None], lam, 1.0))
    out[:, 7] = np.log(np.asarray(rho_cell, np.float64)[members])
    out[:, 8:11] = np.abs(np.einsum("mi,mia->ma", dl, E)) / sl
    siso = np.sqrt(lam.sum(1) / 3.0)
    out[:, 11] = np.linalg.norm(vm.T - vloc, axis=1) / np.where(ok, siso, 1.0)
    out[~ok, 1:] = np.nan
    return out


def normalise(F, shift, scale):
    """(F - shift) * scale per column (the inputs the network sees)."""
    return (np.asarray(F, np.float64) - np.asarray(shift, np.float64)) * np.asarray(scale, np.float64)


# ---- the surrogate + fallback decision ------------------------------------------
def decide(Rhat, R_exact, threshold, margin):
    """Outliers of the surrogate path: inside the band |Rhat - threshold| <
    margin (or Rhat not finite) the exact R decides, outside it Rhat does.
    Returns (outlier mask, band mask)."""
    Rhat = np.asarray(Rhat, np.float64)
    band = ~np.isfinite(Rhat) | (np.abs(Rhat - threshold) < margin)
    out = np.where(band, np.asarray(R_exact, np.float64) >= threshold, Rhat >= threshold)
    return out, band


def recall_precision(pred, truth):
    pred = np.asarray(pred, bool)
    truth = np.asarray(truth, bool)
    tp = np.count_nonzero(pred & truth)
    rec = tp / max(1, np.count_nonzero(truth))
    prec = tp / max(1, np.count_nonzero(pred))
    return rec, prec
