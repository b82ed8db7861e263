"""GPU checks of the surrogate MLP (MFMA, bf16 operands, FP32 accumulation)
against the FP64 reference evaluated on the same bf16-rounded operands, and
of the top-k selection."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu

DIMS = (100, 256, 3, 40)


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


def _rand(seed, B, scale=0.08):
    rng = np.random.default_rng(seed)
    shp = ref.shapes(*DIMS)
    n = sum(r * c + r for r, c in shp)
    theta = rng.normal(0, scale, n).astype(np.float32)
    X = rng.normal(0, 1, (B, DIMS[0])).astype(np.float32)
    T = rng.normal(0, 1, (B, DIMS[3])).astype(np.float32)
    return shp, theta, X, T


@pytest.mark.parametrize("B", [1, 77, 300])
def test_forward_matches_reference_on_rounded_operands(dtb, B):
    shp, theta, X, T = _rand(1, B)
    m = dtb.MLP(*DIMS)
    m.set_params(theta)
    Y = m.forward(X).astype(np.float64)
    Yr, _ = ref.forward(theta.astype(np.float64), X, shp, bf16=True)
    rel = np.linalg.norm(Y - Yr) / np.linalg.norm(Yr)
    assert rel < 1e-3, rel
    Y64, _ = ref.forward(theta.astype(np.float64), X, shp, bf16=False)
    assert np.linalg.norm(Y - Y64) / np.linalg.norm(Y64) < 2e-2


def test_gradient_matches_reference_per_layer(dtb):
    shp, theta, X, T = _rand(2, 256)
    m = dtb.MLP(*DIMS)
    m.set_params(theta)
    loss, g = m.grad(X, T)
    lr_, gr = ref.loss_and_grad(theta.astype(np.float64), X, T, shp, bf16=True)
    assert abs(loss - lr_) <= 1e-4 * abs(lr_)
    o = 0
    for (r, c) in shp:
        for size in (r * c, r):
            a, b = g[o:o + size].astype(np.float64), gr[o:o + size]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            assert rel < 1e-2, (o, size, rel)
            o += size
    _, g64 = ref.loss_and_grad(theta.astype(np.float64), X, T, shp, bf16=False)
    assert np.linalg.norm(g - g64) / np.linalg.norm(g64) < 2e-2


def test_adam_step_matches_reference(dtb):
    shp, theta, X, T = _rand(3, 128)
    m = dtb.MLP(*DIMS)
    m.set_params(theta)
    _, g = m.grad(X, T)
    m.train_step(X, T, lr=1e-3)
    new = m.get_params().astype(np.float64)
    t_ref, _, _ = ref.adam(theta.astype(np.float64), np.zeros(len(theta)), np.zeros(len(theta)),
                           g.astype(np.float64), 1, 1e-3)
    np.testing.assert_allclose(new, t_ref, rtol=0, atol=2e-7 + 1e-6 * np.abs(t_ref).max())


def test_adam_trajectory_matches_reference(dtb):
    """20 Adam steps on the GPU track 20 FP64 reference steps (same bf16
    rounding points): losses and final parameters agree closely."""
    shp, theta, X, T = _rand(8, 256)
    m = dtb.MLP(*DIMS)
    m.set_params(theta)
    th = theta.astype(np.float64)
    mm = np.zeros(len(th))
    vv = np.zeros(len(th))
    for step in range(1, 21):
        lo = m.train_step(X, T, lr=1e-3)
        lr_, g = ref.loss_and_grad(th, X, T, shp, bf16=True)
        assert abs(lo - lr_) <= 2e-3 * abs(lr_), (step, lo, lr_)
        th, mm, vv = ref.adam(th, mm, vv, g, step, 1e-3)
    new = m.get_params().astype(np.float64)
    assert np.linalg.norm(new - th) / np.linalg.norm(th - theta) < 5e-2


def test_training_reduces_loss_on_a_teacher_network(dtb):
    """Regress the outputs of a fixed random 'teacher' network: Adam on the
    MFMA kernels drives the held-in loss down several-fold."""
    shp, teacher, _, _ = _rand(4, 1, scale=0.1)
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (4096, DIMS[0])).astype(np.float32)
    Y, _ = ref.forward(teacher.astype(np.float64), X, shp)
    Y = ((Y - Y.mean(0)) / (Y.std(0) + 1e-12)).astype(np.float32)
    m = dtb.MLP(*DIMS, seed=11)
    first = m.grad(X[:1024], Y[:1024])[0]
    for ep in range(40):
        for b in range(0, 4096, 256):
            m.train_step(X[b:b + 256], Y[b:b + 256], lr=2e-3)
    last = m.grad(X[:1024], Y[:1024])[0]
    assert last < first / 3, (first, last)


def test_topk_is_exact_with_ties_and_nan(dtb):
    rng = np.random.default_rng(6)
    for n, k in [(4096, 64), (1000, 17), (5, 5), (1, 1)]:
        s = rng.integers(0, 50, n).astype(np.float32)  # many ties
        if n > 10:
            s[3] = np.nan
        idx = dtb.topk(s, k)
        key = np.where(np.isnan(s), np.inf, s)
        order = np.lexsort((np.arange(n), key))[:k]
        np.testing.assert_array_equal(idx, order)


def _close_per_tensor(a, b, tol):
    """max over entries of |a - b| / (|b| + mean |b|) <= tol."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    r = float((np.abs(a - b) / (np.abs(b) + np.mean(np.abs(b)))).max())
    assert r <= tol, r
    return r


@pytest.mark.parametrize("B", [256, 77])
def test_fp32_operands_match_unrounded_reference_elementwise(dtb, B):
    """The kernels' logic (tiling, transposes, tails, epilogues, MSE, bias
    sums) with every matrix operand in FP32: the output and every gradient
    entry within 1e-5 of the unrounded FP64 reference, per entry relative
    to |ref| + mean |ref| of its tensor (FP32 arithmetic of the same
    products gives about 2e-6 on this measure).  Switching back to bfloat16
    operands restores the rounded path."""
    shp, theta, X, T = _rand(2, B)
    m = dtb.MLP(*DIMS)
    m.set_params(theta)
    Yb = m.forward(X)
    m.set_operands(True)
    theta64 = theta.astype(np.float64)
    Y64, _ = ref.forward(theta64, X, shp, bf16=False)
    _close_per_tensor(m.forward(X), Y64, 1e-5)
    loss, g = m.grad(X, T)
    l64, g64 = ref.loss_and_grad(theta64, X, T, shp, bf16=False)
    assert abs(loss - l64) <= 1e-5 * abs(l64)
    o = 0
    for (r, c) in shp:
        for size in (r * c, r):
            _close_per_tensor(g[o:o + size], g64[o:o + size], 1e-5)
            o += size
    m.set_operands(False)
    np.testing.assert_array_equal(m.forward(X), Yb)
