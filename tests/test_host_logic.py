"""Host-side logic of the package (no GPU): the surrogate's margin
calibration and scores against the oracle's decision rule."""
import numpy as np
import torch

from oracle import surrogate as S
from paper_1902_01010_amd import surrogate


def test_calibrated_margin_meets_recall_and_is_tight():
    rng = np.random.default_rng(3)
    r_ex = rng.normal(1.0, 1.5, 20000)
    rhat = r_ex + rng.normal(0, 0.6, r_ex.size)
    rhat[::501] = np.nan
    for target in (0.9, 0.99, 0.995):
        mg = surrogate.calibrate_margin(torch.from_numpy(rhat), torch.from_numpy(r_ex), 2.0, target)
        out, band = S.decide(rhat, r_ex, 2.0, mg)
        rec, _ = S.recall_precision(out, r_ex >= 2.0)
        assert rec >= target
        # a slightly smaller margin loses the target
        out2, _ = S.decide(rhat, r_ex, 2.0, mg * 0.98 - 2e-3)
        assert S.recall_precision(out2, r_ex >= 2.0)[0] < target or mg < 1e-3
        sc = surrogate.score(torch.from_numpy(rhat), torch.from_numpy(r_ex), 2.0, mg)
        ref_rec, ref_prec = S.recall_precision(out, r_ex >= 2.0)
        assert sc["recall"] == ref_rec and sc["precision"] == ref_prec
        assert sc["band_frac"] == band.mean()
