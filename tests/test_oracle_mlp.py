"""Pins of the learned-closure reference network (oracle): forward pass on
hand-built weights with a closed form, back-propagated gradient against
central finite differences, bfloat16 rounding on known values, Adam's first
step, and the closure's output mapping and fallback rule."""
import numpy as np
import pytest

NI, NH, NO = 12, 64, 2


def offsets():
    o = {}
    k = 0
    for name, size in (("W1", NH * NI), ("b1", NH), ("W2", NH * NH), ("b2", NH), ("W3", NH * NH), ("b3", NH),
                       ("W4", NO * NH), ("b4", NO)):
        o[name] = (k, size)
        k += size
    assert k == 9282
    return o


def silu(x):
    return x / (1 + np.exp(-x))


def test_forward_closed_form_chain(oracle_lib):
    """A single active path input0 -> h1_0 -> h2_0 -> h3_0 -> o_0 with unit
    weights gives o_0 = silu(silu(silu(x0))) + b4_0 and o_1 = b4_1."""
    O = offsets()
    p = np.zeros(9282)
    p[O["W1"][0] + 0 * NI + 0] = 1.0
    p[O["W2"][0] + 0] = 1.0
    p[O["W3"][0] + 0] = 1.0
    p[O["W4"][0] + 0] = 1.0
    p[O["b4"][0] + 0] = 0.25
    p[O["b4"][0] + 1] = -0.5
    X = np.zeros((3, NI))
    X[:, 0] = [-2.0, 0.3, 4.0]
    out = oracle_lib.mlp_forward(p, X)
    exp0 = silu(silu(silu(X[:, 0]))) + 0.25
    assert np.allclose(out[:, 0], exp0, rtol=1e-15, atol=1e-15)
    assert np.allclose(out[:, 1], -0.5)


def _random_params(seed):
    rng = np.random.default_rng(seed)
    O = offsets()
    p = np.zeros(9282)
    for name, fan in (("W1", NI), ("W2", NH), ("W3", NH), ("W4", NH)):
        a, n = O[name]
        p[a:a + n] = rng.uniform(-1, 1, n) / np.sqrt(fan)
    for name in ("b1", "b2", "b3", "b4"):
        a, n = O[name]
        p[a:a + n] = rng.uniform(-0.1, 0.1, n)
    return p


def test_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(1)
    p = _random_params(2)
    X = rng.normal(size=(7, NI))
    T = rng.normal(size=(7, NO))
    loss, g = oracle_lib.mlp_grad(p, X, T)
    idx = np.concatenate([rng.choice(9282, 60, replace=False), [0, 767, 768, 9279, 9280, 9281]])
    for q in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        lp, _ = oracle_lib.mlp_grad(pp, X, T)
        lm, _ = oracle_lib.mlp_grad(pm, X, T)
        fd = (lp - lm) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-9), q
    # the loss is the mean over samples of the summed squared output error
    o = oracle_lib.mlp_forward(p, X)
    assert loss == pytest.approx(np.sum((o - T) ** 2) / 7, rel=1e-13)


def test_bf16_round_to_nearest_even(oracle_lib):
    b = oracle_lib.bf16
    assert b(1.0) == 1.0
    assert b(1.0 + 2.0 ** -8) == 1.0                     # tie -> even (mantissa ...0)
    assert b(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (rounds up)
    assert b(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert b(-3.14159) == -3.140625
    assert b(65504.0) == 65536.0
    assert b(1e-3) == pytest.approx(1e-3, rel=2 ** -8)


def test_bf16_forward_close_to_fp64(oracle_lib):
    rng = np.random.default_rng(3)
    p = _random_params(4)
    X = rng.normal(size=(256, NI))
    a = oracle_lib.mlp_forward(p, X)
    b = oracle_lib.mlp_forward(p, X, bf16=True)
    rel = np.abs(a - b).max() / np.abs(a).max()
    assert 1e-5 < rel < 5e-2


def test_adam_first_step_moves_by_lr(oracle_lib):
    """With bias correction the first Adam step is lr * g / (|g| + eps)."""
    p = np.linspace(-1, 1, 9282)
    g = np.where(np.arange(9282) % 2, 0.3, -2e-3)
    m = np.zeros(9282)
    v = np.zeros(9282)
    p0 = p.copy()
    oracle_lib.adam_step(p, g, m, v, 1, lr=1e-3)
    assert np.allclose(p0 - p, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _closure_args():
    """Zero network weights with output biases (b0, b1): the raw outputs are
    the biases whatever the inputs.  Unit normalisation, training range
    [-1, 1] on every input."""
    O = offsets()
    p = np.zeros(9282)
    return p, O["b4"][0], np.zeros(NI), np.ones(NI), -np.ones(NI), np.ones(NI)


def test_closure_output_mapping_closed_form(oracle_lib):
    """nu_t = Delta^2 |S| softplus(o_1), Pr_t = 0.1 + softplus(o_2), with
    |S|^2 = 2 S_ij S_ij; softplus(0) = ln 2."""
    p, b4, mean, std, lo, hi = _closure_args()
    gu = np.array([[0.0, 0.0, 0.02], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]) * 0.5   # |S| = 0.01
    Delta = 50.0
    mean[10] = Delta     # the filter-width input at the centre of its range
    for o1, o2 in ((0.0, 0.0), (1.5, -2.0), (-3.0, 4.0), (40.0, 0.3)):
        p[b4], p[b4 + 1] = o1, o2
        fb, nu, pr = oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta, 0.0)
        assert not fb
        sp1 = np.log1p(np.exp(o1)) if o1 < 30 else o1
        assert nu == pytest.approx(Delta ** 2 * 0.01 * sp1, rel=1e-14)
        assert pr == pytest.approx(0.1 + np.log1p(np.exp(o2)), rel=1e-14)
    p[b4], p[b4 + 1] = 0.0, 0.0
    _, nu, pr = oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta, 0.0)
    assert nu == pytest.approx(Delta ** 2 * 0.01 * np.log(2.0), rel=1e-15)
    assert pr == pytest.approx(0.1 + np.log(2.0), rel=1e-15)
    # no strain, no viscosity: the rest state stays at rest
    _, nu0, _ = oracle_lib.mlp_closure(p, mean, std, lo, hi, np.zeros((3, 3)), 0.0, Delta, 0.0)
    assert nu0 == 0.0


def test_closure_fallback_rule(oracle_lib):
    """Fallback when a standardised input leaves [lo, hi] widened by 10 % of
    its half-width (plus the 2^-20 (1 + |mean/std|) rounding margin), or the
    output is not finite; never with the fallback switched off."""
    p, b4, mean, std, lo, hi = _closure_args()
    Delta = 1.0          # input 10 (the filter width): x = 1 with mean 0, std 1
    gu = np.zeros((3, 3))
    for val, expect in ((1.05, False), (-1.09, False), (1.12, True), (-1.2, True)):
        g = gu.copy()
        g[0, 1] = val    # input 1 (du/dy)
        fb, _, _ = oracle_lib.mlp_closure(p, mean, std, lo, hi, g, 0.0, Delta, 0.0)
        assert fb == expect, val
        fb, _, _ = oracle_lib.mlp_closure(p, mean, std, lo, hi, g, 0.0, Delta, 0.0, use_fallback=False)
        assert not fb
    # N^2 (input 9) and the TKE estimate (input 11) are checked too
    assert oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 1.2, Delta, 0.0)[0]
    assert oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta, 0.2)[0]   # (0.2/0.1)^2 = 4
    # a non-finite output falls back
    p[b4] = np.nan
    assert oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta, 0.0)[0]


def test_closure_constant_training_input_passes_at_its_value(oracle_lib):
    """An input that was constant in training (the filter width on a
    uniform mesh: half-width 0, std set to 1) passes when it equals the
    float-rounded training mean, also for a width that float cannot hold
    exactly, and falls back when it moves off that value."""
    p, b4, mean, std, lo, hi = _closure_args()
    Delta = 1000.0 / 12.0                      # 83.333..., not a float
    mean[10] = float(np.float32(Delta))
    lo[10] = hi[10] = 0.0
    gu = np.zeros((3, 3))
    assert not oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta, 0.0)[0]
    assert oracle_lib.mlp_closure(p, mean, std, lo, hi, gu, 0.0, Delta * 1.001, 0.0)[0]


def test_bf16_emulated_gradient_against_fp64(oracle_lib):
    """The gradient with the GPU's rounding points (bfloat16 products, FP32
    sums and activations) stays within the bfloat16 rounding of the FP64
    back-propagated gradient (pinned above by finite differences), term by
    term: |g16 - g64| <= 0.03 sum|terms|, with 2^-8 the bfloat16 unit
    roundoff compounded over four layers. A dropped term, a transposed
    operand or a derivative at the wrong layer is an O(1) change of that
    ratio. Its loss is the mean squared error of the bfloat16 forward pass."""
    rng = np.random.default_rng(6)
    p = _random_params(7).astype(np.float32).astype(np.float64)
    X = rng.normal(size=(300, NI)).astype(np.float32).astype(np.float64)
    T = rng.normal(size=(300, NO)).astype(np.float32).astype(np.float64)
    l64, g64 = oracle_lib.mlp_grad(p, X, T)
    l16, g16, mag = oracle_lib.mlp_grad_bf16(p, X, T)
    assert np.all(mag > 0)
    ratio = np.abs(g16 - g64) / mag
    assert ratio.max() < 0.03, ratio.max()
    assert np.linalg.norm(g16 - g64) < 1e-2 * np.linalg.norm(g64)
    # and it is not the FP64 gradient: the rounding shows
    assert ratio.max() > 1e-5
    o16 = oracle_lib.mlp_forward(p, X, bf16=True)
    assert l16 == pytest.approx(np.sum((o16 - T) ** 2) / 300, rel=1e-6)
    assert l16 == pytest.approx(l64, rel=1e-2)
