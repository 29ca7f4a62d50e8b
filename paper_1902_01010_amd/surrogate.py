"""Training, calibration and storage of the learned R surrogate.

The network (12 features -> 64 -> 64 -> 64 -> 1, ReLU) is trained on the GPU
by the library's own kernels (vr_mlp_train_step: BF16 MFMA forward and
backward, FP32 Adam) on the exact R that the plain path computes for the
searched particles of several synthetic boxes.  The band margin is then set
on a held-out box so that the surrogate+fallback path keeps at least the
target recall of the exact path's outliers, and frozen.

Usage (on a GPU):  python -m paper_1902_01010_amd.surrogate --out MODEL.npz
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import pipeline, synth
from . import vr as _vr

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "surrogate_model.npz")
TARGET_CLIP = (-6.0, 10.0)   # only the order around the threshold matters


@dataclasses.dataclass
class SurrogateModel:
    weights: torch.Tensor          # device FP32 [MLP_PARAMS]
    shift: np.ndarray              # 12 feature shifts
    scale: np.ndarray              # 12 feature scales
    margin: float                  # band half-width around the threshold
    cell_scale: float = 0.5        # fine feature cell side as a fraction of ellx (rounded down to 2^k units)
    cell_bits: int = 0             # set per box by bind()
    meta: dict = dataclasses.field(default_factory=dict)

    def bind(self, prm: pipeline.Params, box: float, grid_bits: int) -> "SurrogateModel":
        """The model with the feature cell size of a box (same physical size everywhere)."""
        ell_grid = prm.ellx * 2.0 ** grid_bits / box
        cb = int(math.floor(math.log2(ell_grid * self.cell_scale)))
        cb = max(0, min(cb, grid_bits - 4))
        return dataclasses.replace(self, cell_bits=cb)

    def save(self, path):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, weights=self.weights.detach().cpu().numpy().astype(np.float32),
                 shift=np.asarray(self.shift, np.float32), scale=np.asarray(self.scale, np.float32),
                 margin=np.float64(self.margin), cell_scale=np.float64(self.cell_scale),
                 meta=np.array(json.dumps(self.meta)))

    @classmethod
    def load(cls, path=MODEL_PATH, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            return cls(weights=torch.from_numpy(z["weights"].copy()).to(device), shift=z["shift"].copy(),
                       scale=z["scale"].copy(), margin=float(z["margin"]), cell_scale=float(z["cell_scale"]),
                       meta=json.loads(str(z["meta"])))


def exact_box(ctx, seed, n_side):
    """A synthetic box through the plain path up to R (device outputs)."""
    w = synth.cosmo_box(seed=seed, n_side=n_side)
    prm = pipeline.Params.from_workload(w)
    x, v, m = pipeline.device_inputs(w)
    out, _ = pipeline.run(ctx, x, v, m, w.mass_value, w.box, w.grid_bits, prm, until="R")
    return w, prm, out


def box_features(ctx, w, prm, out, cell_bits, shift=None, scale=None):
    P = _vr.Particles(out["q"], torch.from_numpy(w.v).cuda(), None if w.mass is None else torch.from_numpy(w.mass).cuda(),
                      w.mass_value, w.box, w.grid_bits)
    cm = out["cells"]
    feat = ctx.rs_features(P, out["host_offsets"], out["members"], cm["vbar"], cm["sigma"], cm["rho_cell"], prm.n_se,
                           cell_bits, shift, scale)
    rows = out["members"][:feat.shape[0]].long()
    return feat, out["R"][rows]


def bf16_to_float(feat):
    return ((feat.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)


def calibrate_margin(rhat, r_exact, threshold, recall):
    """Smallest margin for which the outliers the band misses (exact R >=
    threshold, Rhat <= threshold - margin) stay within 1 - recall."""
    rh = rhat.double().cpu().numpy()
    re = r_exact.double().cpu().numpy()
    truth = re >= threshold
    d = threshold - rh[truth & np.isfinite(rh)]
    allowed = int(math.floor((1.0 - recall) * truth.sum()))
    d = np.sort(d)[::-1]
    if len(d) == 0:
        return 0.0
    k = min(allowed, len(d) - 1)
    return float(max(d[k], 0.0) * (1 + 1e-6) + 1e-4)


def score(rhat, r_exact, threshold, margin):
    """Recall and precision of the surrogate+fallback outliers against the
    exact ones, the band fraction, and the band each recall level needs."""
    rh = rhat.double().cpu().numpy()
    re = r_exact.double().cpu().numpy()
    band = ~np.isfinite(rh) | (np.abs(rh - threshold) < margin)
    pred = np.where(band, re >= threshold, rh >= threshold)
    truth = re >= threshold
    tp = np.count_nonzero(pred & truth)
    curve = {}
    for rec in (0.9, 0.95, 0.99, 0.995):
        mg = calibrate_margin(rhat, r_exact, threshold, rec)
        curve[str(rec)] = float((~np.isfinite(rh) | (np.abs(rh - threshold) < mg)).mean())
    return dict(recall=tp / max(1, truth.sum()), precision=tp / max(1, pred.sum()), band_frac=float(band.mean()),
                outliers=int(truth.sum()), rows=int(len(re)), band_for_recall=curve)


def train(ctx, train_seeds=range(401, 409), calib_seed=409, n_side=128, epochs=20, batch=8192, lr=2e-3,
          recall=0.995, init_seed=7, log=print):
    t0 = time.time()
    boxes = []
    for s in train_seeds:
        w, prm, out = exact_box(ctx, s, n_side)
        boxes.append((w, prm, out))
        log(f"[surrogate] box seed {s}: {out['n_searched']} searched particles ({time.time() - t0:.0f} s)")
    base = SurrogateModel(weights=None, shift=np.zeros(12), scale=np.ones(12), margin=0.0)
    # feature statistics from the raw features
    raws = []
    for w, prm, out in boxes:
        mb = base.bind(prm, w.box, w.grid_bits)
        f, _ = box_features(ctx, w, prm, out, mb.cell_bits)
        raws.append(bf16_to_float(f))
    raw = torch.cat(raws)
    ok = torch.isfinite(raw).all(1)
    mu = raw[ok].double().mean(0)
    sd = raw[ok].double().std(0).clamp_min(1e-6)
    shift = mu.cpu().numpy().astype(np.float32)
    scale = (1.0 / sd).cpu().numpy().astype(np.float32)
    del raws, raw
    feats, targets = [], []
    for w, prm, out in boxes:
        mb = base.bind(prm, w.box, w.grid_bits)
        f, r = box_features(ctx, w, prm, out, mb.cell_bits, shift, scale)
        good = torch.isfinite(r) & torch.isfinite(bf16_to_float(f)).all(1)
        feats.append(f[good])
        targets.append(r[good].clamp(*TARGET_CLIP))
    X = torch.cat(feats).contiguous()
    Y = torch.cat(targets).contiguous().float()
    del boxes, feats, targets
    n = X.shape[0]
    log(f"[surrogate] {n} training rows; outlier fraction {(Y >= 2.0).float().mean().item():.4f}")
    wts = torch.from_numpy(synth.mlp_init(init_seed)).cuda()
    st = torch.zeros(2 * _vr.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(init_seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen).to(torch.int32)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        for b in range(steps_per_epoch):
            step += 1
            # cosine decay from lr to lr / 20
            lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total)))
            ctx.mlp_train_step(wts, st, X, Y, step, rows=perm[b * batch:(b + 1) * batch], lr=lr_t, loss=loss)
            acc += loss
        log(f"[surrogate] epoch {ep + 1}/{epochs}: mean batch loss {acc.item() / steps_per_epoch:.4f} "
            f"({time.time() - t0:.0f} s)")
    model = SurrogateModel(weights=wts, shift=shift, scale=scale, margin=0.0)
    # the band margin, on a held-out box, then frozen
    w, prm, out = exact_box(ctx, calib_seed, n_side)
    mb = model.bind(prm, w.box, w.grid_bits)
    f, r = box_features(ctx, w, prm, out, mb.cell_bits, shift, scale)
    rhat = ctx.mlp_forward(wts, f)
    model.margin = calibrate_margin(rhat, r, prm.R_threshold, recall)
    sc = score(rhat, r, prm.R_threshold, model.margin)
    model.meta = dict(train_seeds=list(train_seeds), calib_seed=calib_seed, n_side=n_side, epochs=epochs,
                      batch=batch, lr=lr, init_seed=init_seed, rows=n, recall_target=recall, calib=sc,
                      final_loss=float(loss.item()))
    log(f"[surrogate] margin {model.margin:.4f} on seed {calib_seed}: {json.dumps(sc)} ({time.time() - t0:.0f} s)")
    return model


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--n-side", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--train-seeds", default="401-408")
    ap.add_argument("--calib-seed", type=int, default=409)
    args = ap.parse_args()
    a, b = (int(t) for t in args.train_seeds.split("-"))
    ctx = _vr.Context(0)
    model = train(ctx, range(a, b + 1), args.calib_seed, args.n_side, args.epochs, args.batch, args.lr,
                  log=lambda s: print(s, flush=True))
    model.save(args.out)
    print(f"[surrogate] saved {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
