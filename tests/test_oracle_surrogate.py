"""Pins of the surrogate oracle (features, MLP, gradients, Adam) against
closed forms, brute force and independent library routines."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_1902_01010_amd import synth


# ---- BF16 rounding ---------------------------------------------------------------
def test_bf16_round_ties_to_even_and_matches_torch():
    one = 1.0
    assert S.bf16_round(one) == 1.0
    assert S.bf16_round(1 + 2.0 ** -8) == 1.0                    # midpoint, even neighbour below
    assert S.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6      # midpoint, even neighbour above
    assert S.bf16_round(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, np.inf, -np.inf, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16_round(x), ref)
    assert np.isnan(S.bf16_round(np.float32(np.nan)))
    np.testing.assert_array_equal(S.bf16_from_bits(S.bf16_bits(x)), ref)


# ---- MLP ------------------------------------------------------------------------------
def _abs_net(b4=0.25):
    W1 = np.zeros((12, 64)); W1[0, 0] = 1.0; W1[0, 1] = -1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = W2[1, 1] = 1.0
    W3 = np.zeros((64, 64)); W3[0, 0] = W3[1, 1] = 1.0
    w4 = np.zeros(64); w4[0] = w4[1] = 1.0
    return S.pack([W1, np.zeros(64), W2, np.zeros(64), W3, np.zeros(64), w4, [b4]])


def test_mlp_forward_closed_form_abs():
    """ReLU(x) + ReLU(-x) = |x|: a network that must output |x_0| + b4."""
    w = _abs_net()
    X = np.zeros((7, 12))
    X[:, 0] = [-3.0, -1.5, -0.25, 0.0, 0.5, 2.0, 7.0]        # BF16-exact values
    X[:, 5] = 100.0                                           # ignored input
    for bf in (False, True):
        np.testing.assert_array_equal(S.forward(w, X, bf16=bf), np.abs(X[:, 0]) + 0.25)


def test_mlp_forward_bias_only_and_unpack_layout():
    w = np.zeros(S.MLP_PARAMS)
    W1, b1, W2, b2, W3, b3, w4, b4 = S.unpack(w)
    assert W1.shape == (12, 64) and W3.shape == (64, 64) and w4.shape == (64,) and b4.shape == (1,)
    assert S.MLP_PARAMS == 9217
    parts = [np.zeros((12, 64)), np.full(64, 0.5), np.zeros((64, 64)), np.full(64, -1.0),
             np.eye(64), np.full(64, 2.0), np.full(64, 0.125), [1.0]]
    # layer 2 output is ReLU(-1) = 0, so layer 3 is ReLU(0 + 2) = 2 everywhere
    y = S.forward(S.pack(parts), np.random.default_rng(0).normal(size=(5, 12)), bf16=False)
    np.testing.assert_allclose(y, 64 * 2.0 * 0.125 + 1.0)


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    w = synth.mlp_init(11).astype(np.float64)
    w[12 * 64:12 * 64 + 64] = rng.normal(scale=0.1, size=64)       # non-zero biases
    X = rng.normal(size=(24, 12))
    y = rng.normal(size=24)
    loss, g = S.loss_and_grad(w, X, y)
    assert loss == pytest.approx(np.mean((S.forward(w, X, bf16=False) - y) ** 2), rel=1e-12)
    idx = rng.choice(S.MLP_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [S.MLP_PARAMS - 1, S.MLP_PARAMS - 2, 0, 12 * 64]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(w); e[i] = h
        num = (S.loss_and_grad(w + e, X, y)[0] - S.loss_and_grad(w - e, X, y)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_mlp_gradient_rounded_model_is_exact_on_representable_values():
    """With small-integer weights, inputs and targets, sparse hidden layers and
    a power-of-two batch, every operand the rounded model rounds (weights,
    activations, errors) is already a BF16 number, so the model must equal the
    exact gradient bit for bit."""
    rng = np.random.default_rng(12)
    parts = [rng.integers(-1, 2, (12, 64)), rng.integers(-2, 3, 64), rng.integers(-1, 2, (64, 64)) * (rng.random((64, 64)) < 0.05),
             rng.integers(-2, 3, 64), rng.integers(-1, 2, (64, 64)) * (rng.random((64, 64)) < 0.05),
             rng.integers(-2, 3, 64), rng.integers(-1, 2, 64), [1.0]]
    w = S.pack(parts)
    X = rng.integers(-3, 4, (16, 12)).astype(float)
    y = rng.integers(-8, 9, 16).astype(float)
    l0, g0 = S.loss_and_grad(w, X, y)
    l1, g1 = S.loss_and_grad(w, X, y, bf16=True)
    assert np.abs(g0).max() > 0
    assert l0 == l1
    np.testing.assert_array_equal(g0, g1)


def test_mlp_gradient_rounded_model_close_to_exact():
    rng = np.random.default_rng(13)
    w = synth.mlp_init(14).astype(np.float64)
    X = rng.normal(size=(200, 12))
    y = rng.normal(size=200)
    _, g0 = S.loss_and_grad(w, S.bf16_round(X), y)
    _, g1 = S.loss_and_grad(w, X, y, bf16=True)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 5e-2
    assert not np.array_equal(g0, g1)


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(2)
    w0 = rng.normal(size=50)
    g = rng.normal(size=50)
    lr = 1e-3
    w1, m1, m2 = S.adam_step(w0, np.zeros(50), np.zeros(50), g, 1, lr)
    # first step: bias-corrected moments are g and g^2
    np.testing.assert_allclose(w1, w0 - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # several steps against torch's Adam (FP64 on the CPU)
    p = torch.tensor(w0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    w, a, b = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        gt = rng.normal(size=50)
        p.grad = torch.tensor(gt)
        opt.step()
        w, a, b = S.adam_step(w, a, b, gt, t, lr)
    np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-15)


# ---- features ----------------------------------------------------------------------
def _lattice(gb=9, a=16):
    k = np.arange(0, 1 << gb, a)
    g = np.stack(np.meshgrid(k, k, k, indexing="ij"), 0).reshape(3, -1).astype(np.uint32)
    return g


def _iso_inputs(n, rng, lam=(1.0, 4.0, 9.0)):
    vbar = rng.normal(size=(3, n)) * 10
    sig = np.zeros((6, n))
    sig[0], sig[1], sig[2] = lam
    return vbar, sig


@pytest.mark.parametrize("n_se,expect_level", [(32, "fine"), (250, "coarse")])
def test_features_density_on_a_lattice(n_se, expect_level):
    """Particles on a full periodic lattice of spacing a: every window sees
    number density 1/a^3, so rhat = (3 n_se / (4 pi))^(1/3) a exactly."""
    gb, a, box = 9, 16, 3.0
    q = _lattice(gb, a)
    n = q.shape[1]
    rng = np.random.default_rng(3)
    v = rng.normal(size=(3, n))
    vbar, sig = _iso_inputs(n, rng)
    rho = np.full(n, 7.0)
    F = S.features(q, v, np.arange(n), vbar, sig, rho, n_se, 5, box, gb)
    unit = box / 2 ** gb
    np.testing.assert_allclose(F[:, 0], np.log((3 * n_se / (4 * np.pi)) ** (1 / 3) * a * unit), rtol=1e-12)
    np.testing.assert_allclose(F[:, 7], np.log(7.0))
    # 27 fine cells of side 32 hold 27 * 8 = 216 lattice points
    assert (216 >= n_se) == (expect_level == "fine")


def test_features_counts_against_brute_force():
    """The window counts and the face-neighbour mean velocity, recomputed by
    a plain loop over all pairs of members (periodic cell distance)."""
    gb, c, box = 10, 5, 1.0
    rng = np.random.default_rng(4)
    n = 900
    q = np.empty((3, n), np.uint32)
    q[:, :600] = (rng.normal(size=(3, 600)) * 60 + 100).astype(np.int64) % (1 << gb)
    q[:, 600:] = rng.integers(0, 1 << gb, (3, 300))
    q[:, 0] = [3, 1020, 512]                                   # near the periodic edges
    v = rng.normal(size=(3, n)) * 50
    members = np.sort(rng.choice(n, 700, replace=False))
    vbar, sig = _iso_inputs(n, rng)
    rho = np.ones(n)
    n_se = 20
    F = S.features(q, v, members, vbar, sig, rho, n_se, c, box, gb)
    unit = box / 2 ** gb
    qm = q[:, members].astype(np.int64)

    def cdist(cb):
        cc = qm >> cb
        nc = 1 << (gb - cb)
        d = np.abs(cc[:, :, None] - cc[:, None, :])
        return np.minimum(d, nc - d)                              # 3 x m x m

    dfine, dcoarse = cdist(c), cdist(c + 2)
    nf = (dfine.max(0) <= 1).sum(1)
    ncs = (dcoarse.max(0) <= 1).sum(1)
    f = 2.0 ** c * unit
    nhat = np.where(nf >= n_se, nf / (27 * f ** 3), ncs / (27 * (4 * f) ** 3))
    np.testing.assert_allclose(F[:, 0], np.log((3 * n_se / (4 * np.pi * nhat)) ** (1 / 3)), rtol=1e-12)
    assert (nf >= n_se).any() and (nf < n_se).any()
    face = dfine.sum(0) <= 1                                      # own cell or one face step
    vm = v[:, members]
    vloc = (face.astype(float) @ vm.T) / face.sum(1)[:, None]
    np.testing.assert_allclose(F[:, 11], np.linalg.norm(vm.T - vloc, axis=1) / np.sqrt(14 / 3), rtol=1e-10)


def test_features_rotation_invariance_and_eigen_closed_form():
    rng = np.random.default_rng(6)
    n = 200
    q = rng.integers(0, 1 << 12, (3, n)).astype(np.uint32)
    lam = np.array([0.5, 3.0, 20.0])
    coef = rng.normal(size=(n, 3))
    F0 = None
    for trial in range(4):
        Rm, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        Sig = Rm @ np.diag(lam) @ Rm.T
        sig = np.tile(np.array([Sig[0, 0], Sig[1, 1], Sig[2, 2], Sig[0, 1], Sig[0, 2], Sig[1, 2]])[:, None], (1, n))
        vbar = rng.normal(size=(3, n)) * 5
        dv = (coef * np.sqrt(lam)) @ Rm.T                         # components along the eigenvectors
        v = vbar + dv.T
        F = S.features(q, v, np.arange(n), vbar, sig, np.ones(n), 8, 6, 10.0, 12)
        np.testing.assert_allclose(F[:, 1:4], np.abs(coef), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(F[:, 4:7], np.tile(np.log(lam), (n, 1)), rtol=1e-12)
        if F0 is not None:
            np.testing.assert_allclose(F[:, [0, 1, 2, 3, 4, 5, 6, 7]], F0[:, [0, 1, 2, 3, 4, 5, 6, 7]], rtol=1e-9)
        F0 = F


def test_features_uniform_flow_and_non_positive_definite():
    rng = np.random.default_rng(8)
    n = 300
    q = rng.integers(0, 1 << 11, (3, n)).astype(np.uint32)
    v = np.tile(np.array([[100.0], [-20.0], [5.0]]), (1, n))     # every member moves alike
    vbar, sig = _iso_inputs(n, rng)
    sig[:, 7] = [1.0, 1.0, -1.0, 0, 0, 0]                         # not positive definite
    F = S.features(q, v, np.arange(n), vbar, sig, np.ones(n), 8, 5, 1.0, 11)
    ok = np.arange(n) != 7
    np.testing.assert_allclose(F[ok, 11], 0.0, atol=1e-12)
    np.testing.assert_allclose(F[ok, 8:11], F[ok, 1:4], rtol=1e-12)
    assert np.isnan(F[7, 1:]).all() and np.isfinite(F[7, 0])


# ---- decision and scores ----------------------------------------------------------
def test_decide_band_and_scores():
    Rhat = np.array([0.0, 1.95, 2.04, 3.0, np.nan, 2.0])
    Rex = np.array([2.5, 2.1, 1.9, 1.0, 2.2, 2.0])
    out, band = S.decide(Rhat, Rex, 2.0, 0.1)
    np.testing.assert_array_equal(band, [False, True, True, False, True, True])
    np.testing.assert_array_equal(out, [False, True, False, True, True, True])
    rec, prec = S.recall_precision(out, Rex >= 2.0)
    assert rec == pytest.approx(3 / 4) and prec == pytest.approx(3 / 4)   # misses 0, flags 3 wrongly
