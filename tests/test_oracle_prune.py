"""Pins of the oracle's learned-pruning part: number formats, features, the
network's forward pass, loss and gradients, Adam, trace sampling, and the
gated synchronous phase.  Every check compares with something other than
the oracle's own formula: a library routine, a closed form, finite
differences, or a reduction to the plain synchronous phase."""
import math

import numpy as np
import pytest
import torch

import gsp_inputs as gi
import oracle

P = oracle.MLP_PARAMS
W1, B1, W2, B2, W3, B3 = 0, 512, 576, 4672, 4736, 4800


def _rand_params(seed, scale=1.0):
    u = gi.uniform(seed, P)
    p = ((u * 2.0 - 1.0) * scale).astype(np.float32)
    p[W1:B1] *= math.sqrt(6 / 8)
    p[W2:B2] *= math.sqrt(6 / 64)
    p[W3:B3] *= math.sqrt(6 / 64)
    return p


def _rand_rows(seed, rows):
    x = gi.uniform(seed, rows * 8).reshape(rows, 8).astype(np.float32)
    y = (gi.uniform(seed + 1, rows) < 0.4).astype(np.uint8)
    return x, y


# ---------------------------------------------------------------- formats

def test_bf16_matches_torch():
    """bf16 rounding equals torch's float32 -> bfloat16 conversion (round to
    nearest even), including exact ties and values near overflow."""
    u = gi.uniform(3, 4000)
    vals = np.concatenate([
        ((u - 0.5) * 1e4).astype(np.float32),
        ((u - 0.5) * 1e-3).astype(np.float32),
        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0e38, 1e-40, 0.0, -0.0], np.float32),
    ])
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = oracle.bf16(vals)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_plog2_exact_at_powers_and_linear_between():
    for e in range(0, 40):
        assert oracle.plog2(2.0 ** e) == float(e)
        assert oracle.plog2(1.5 * 2.0 ** e) == e + 0.5
    xs = [1 + k for k in range(200)]
    ys = [oracle.plog2(x) for x in xs]
    assert all(b > a for a, b in zip(ys, ys[1:]))
    assert oracle.plog2(0.5) == 0.0


def test_gate_features_values():
    # deg 3 -> plog2(4) / 16 = 0.125; pass 2 -> 0.25; iteration 5 -> 0.25;
    # moved at its last scan -> 1; D = 1.5 of K = 6 -> 0.25
    x = oracle.gate_features(3, 6.0, 24.0, 0.5, -0.25, 3, 1.5, 2, 5)
    assert list(x) == [0.125, 0.5, -0.25, 0.25, 0.25, 0.25, 1.0, 0.25]
    # stayed at its last scan -> 1/2; D above K is capped at 1
    x = oracle.gate_features(3, 6.0, 24.0, 0.5, -0.25, 1, 9.0, 2, 5)
    assert x[6] == 0.5 and x[7] == 1.0
    # capped pass and iteration, isolated vertex, never scanned
    x = oracle.gate_features(0, 0.0, 0.0, 0.0, 0.0, 0, 0.0, 30, 99)
    assert list(x) == [0.0, 0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0]
    # values are bf16: 1/3 rounds to the bf16 nearest
    x = oracle.gate_features(0, 3.0, 9.0, 0.0, 0.0, 0, 1.0, 0, 0)
    third = torch.tensor(1.0 / 3.0, dtype=torch.float32).to(torch.bfloat16).float().item()
    assert x[5] == third and x[7] == third


# ---------------------------------------------------------------- forward

def test_forward_closed_forms():
    x, _ = _rand_rows(5, 50)
    p = np.zeros(P, np.float32)
    p[B3] = 0.75
    assert np.all(oracle.mlp_logits(p, x) == 0.75)            # no weights: the output bias
    p[B2:W3] = np.linspace(-1, 1, 64, dtype=np.float32)       # W2 = 0: constant hidden layer
    p[W3:B3] = np.linspace(0.5, -0.5, 64, dtype=np.float32)
    want = 0.75 + float(np.dot(p[W3:B3].astype(np.float64), np.maximum(p[B2:W3].astype(np.float64), 0.0)))
    assert np.allclose(oracle.mlp_logits(p, x), want, rtol=0, atol=1e-12)


def test_forward_reduces_to_linear_model():
    """W1 = W2 = identity on the first 8 units, x >= 0: z = v . x + b3."""
    x, _ = _rand_rows(6, 64)
    p = np.zeros(P, np.float32)
    for f in range(8):
        p[W1 + f * 8 + f] = 1.0
        p[W2 + f * 64 + f] = 1.0
    v = np.array([0.5, -1.0, 2.0, 0.25, -0.75, 1.5, -2.0, 1.0], np.float32)
    p[W3:W3 + 8] = v
    p[B3] = -0.125
    want = x.astype(np.float64) @ v.astype(np.float64) - 0.125
    assert np.allclose(oracle.mlp_logits(p, x), want, rtol=0, atol=1e-12)
    # a negative first layer is cut by the ReLU: z = b3
    p[W1:B1] *= -1.0
    assert np.allclose(oracle.mlp_logits(p, x[x.min(axis=1) > 0]), -0.125, rtol=0, atol=0)


def test_bf16_formats_exact_on_representable_values():
    """Weights that bf16 holds exactly and small-integer activations: the
    inference formats change nothing."""
    g = gi.uniform(8, P)
    p = (np.round((g - 0.5) * 8) / 8).astype(np.float32)       # multiples of 1/8 in [-0.5, 0.5]
    p[B1:W2] = 0.0
    p[B2:W3] = 0.0
    x = np.round(gi.uniform(9, 40 * 8).reshape(40, 8) * 4).astype(np.float32)
    # first-layer outputs are multiples of 1/8 below 2^5: exact in bf16
    a = oracle.mlp_logits(p, x, bf16_formats=False)
    b = oracle.mlp_logits(p, x, bf16_formats=True)
    assert np.array_equal(a, b)
    # and with general weights the two differ only by bf16 rounding
    p2 = _rand_params(10)
    a, b = oracle.mlp_logits(p2, x), oracle.mlp_logits(p2, x, bf16_formats=True)
    assert np.max(np.abs(a - b)) < 0.05 * (1 + np.max(np.abs(a)))


# ---------------------------------------------------------------- loss, grads

def test_loss_at_zero_logit():
    x, y = _rand_rows(11, 100)
    p = np.zeros(P, np.float32)
    for pw in (1.0, 2.5):
        loss, g = oracle.mlp_loss_grad(p, x, y, pw)
        assert math.isclose(loss, math.log(2.0) * float(np.mean(pw * y + 1 - y)), rel_tol=1e-14)
        # dL/db3 = mean(sigmoid(0) (pw y + 1 - y) - pw y); hidden weights get none
        assert math.isclose(g[B3], float(np.mean(0.5 * (pw * y + 1 - y) - pw * y)), rel_tol=1e-12, abs_tol=1e-15)
        assert np.all(g[:W3] == 0.0)


def test_gradient_matches_central_differences():
    """Central finite differences in fp64 (h = 1e-6) agree with the analytic
    gradient within 1e-6 relative, on parameters from every block.  The
    absolute floor 3e-10 is the rounding of the loss difference itself:
    eps * |L| / h with |L| ~ 1."""
    x, y = _rand_rows(12, 64)
    p = _rand_params(13).astype(np.float64)
    _, g = oracle.mlp_loss_grad_f64(p, x, y, 1.7)
    picks = np.concatenate([np.arange(0, 512, 37), np.arange(512, 576, 7), np.arange(576, 4672, 211),
                            np.arange(4672, 4736, 9), np.arange(4736, 4800, 11), [4800]])
    h = 1e-6
    bad = []
    for k in picks:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (oracle.mlp_loss_grad_f64(pp, x, y, 1.7)[0] - oracle.mlp_loss_grad_f64(pm, x, y, 1.7)[0]) / (2 * h)
        if not math.isclose(fd, g[k], rel_tol=1e-6, abs_tol=3e-10):
            bad.append((int(k), fd, float(g[k])))
    assert not bad, bad[:5]
    assert np.count_nonzero(g[picks]) > 0.8 * len(picks)


def test_fp32_gradient_close_to_fp64():
    x, y = _rand_rows(14, 256)
    p = _rand_params(15)
    l64, g64 = oracle.mlp_loss_grad(p, x, y, 2.0)
    l32, g32 = oracle.mlp_loss_grad(p, x, y, 2.0, fp32=True)
    assert math.isclose(l32, l64, rel_tol=1e-5)
    assert np.linalg.norm(g32 - g64) <= 1e-5 * np.linalg.norm(g64)


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step moves each parameter by
    -lr g / (|g| + eps)."""
    x, y = _rand_rows(16, 128)
    p = _rand_params(17)
    _, g = oracle.mlp_loss_grad(p, x, y, 1.0)
    lr = 1e-3
    p1, _ = oracle.mlp_train_adam(p, x, y, batch=128, epochs=1, lr=lr)
    want = p.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, want.astype(np.float32), rtol=0, atol=2e-7 + 1e-7 * np.abs(p).max())


def _adam_by_hand(b3, batches, pw, lr, epochs):
    """Adam on the output bias alone, written out: with every weight zero
    the network's logit is b3 for every row, so the gradient of the mean
    pos-weighted BCE is [pw P (sigmoid(z) - 1) + N sigmoid(z)] / B for a
    batch of P positive and N negative rows (the other parameters' gradients
    are 0 and they never move).  The gradient is taken at b3 rounded to
    fp32 (the network's storage format).  Returns (b3, per-epoch losses)."""
    m = v = 0.0
    t = 0
    losses = []
    for _ in range(epochs):
        ls = []
        for P, N in batches:
            z = float(np.float32(b3))
            s = 1.0 / (1.0 + math.exp(-z))
            B = P + N
            g = (pw * P * (s - 1.0) + N * s) / B
            ls.append((pw * P * math.log1p(math.exp(-z)) + N * math.log1p(math.exp(z))) / B)
            t += 1
            m = 0.9 * m + 0.1 * g
            v = 0.999 * v + 0.001 * g * g
            b3 -= lr * (m / (1.0 - 0.9 ** t)) / (math.sqrt(v / (1.0 - 0.999 ** t)) + 1e-8)
        losses.append(sum(ls) / len(ls))
    return b3, losses


@pytest.mark.parametrize("batches,epochs,lr", [([(30, 70)], 3, 0.3), ([(10, 54), (50, 14)], 2, 0.05),
                                               ([(3, 125)], 5, 1.0)])
def test_adam_steps_by_hand(batches, epochs, lr):
    """Several Adam steps (moments, bias correction at every t, t counted
    over the batches in order) against the update written out by hand."""
    rows = []
    for P, N in batches:
        rows += [1] * P + [0] * N
    y = np.array(rows, dtype=np.uint8)
    x = gi.uniform(40, y.shape[0] * 8).reshape(-1, 8).astype(np.float32)
    p = np.zeros(oracle.MLP_PARAMS, np.float32)
    p[-1] = 0.25
    pw = 1.5
    want, wl = _adam_by_hand(0.25, batches, pw, lr, epochs)
    got, el = oracle.mlp_train_adam(p, x, y, batch=batches[0][0] + batches[0][1], epochs=epochs, lr=lr,
                                    pos_weight=pw)
    assert np.count_nonzero(got[:-1]) == 0
    assert got[-1] == np.float32(want)
    np.testing.assert_allclose(el, wl, rtol=1e-12)
    # a bias correction missing from the later steps would land far away
    assert abs(want - 0.25) > 10 * abs(float(np.float32(want)) - want)


def test_training_learns_a_separable_rule():
    """Labels y = [x0 + x1 > 1]: Adam drives the loss down and the network
    classifies held-out rows."""
    x = gi.uniform(18, 6000 * 8).reshape(6000, 8).astype(np.float32)
    y = (x[:, 0] + x[:, 1] > 1.0).astype(np.uint8)
    p0 = _rand_params(19)
    p, el = oracle.mlp_train_adam(p0, x[:5000], y[:5000], batch=100, epochs=6, lr=3e-3)
    assert el[-1] < 0.5 * el[0]
    z = oracle.mlp_logits(p, x[5000:])
    acc = np.mean((z >= 0) == (y[5000:] == 1))
    assert acc > 0.95


# ---------------------------------------------------------------- traces

def test_trace_keep_is_splitmix64():
    """mix64 is SplitMix64's output step: seed 1234567 gives the generator's
    published first output 6457827717110365317."""
    first = 6457827717110365317
    assert not oracle.trace_keep(1234567, 0, 0, 0, first)
    assert oracle.trace_keep(1234567, 0, 0, 0, first + 1)


# ---------------------------------------------------------------- gated phase

def test_gated_without_params_is_the_plain_phase():
    g = gi.planted_sbm_10k()
    m, li, dq, mv, cnt = oracle.move_sync_gated(g, None, tau=1e-2)
    m2, li2, dq2, mv2 = oracle.move_sync(g, tau=1e-2)
    assert li == li2 and np.array_equal(m, m2) and np.array_equal(dq, dq2) and np.array_equal(mv, mv2)
    assert cnt["pruned"] == 0 and cnt["confirm_sweeps"] == 0


@pytest.mark.parametrize("make", [lambda: gi.planted_sbm_10k(), lambda: gi.dcsbm_small(6000, 2)])
def test_gate_that_prunes_everything_defers_to_the_confirming_sweep(make):
    """A gate that rejects every vertex: the first gated iteration scans
    nothing, the confirming sweep is the plain phase's first iteration, and
    the plain iterations that follow give the plain phase's result."""
    g = make()
    p = np.zeros(P, np.float32)
    p[B3] = -30.0
    m, li, dq, mv, cnt = oracle.move_sync_gated(g, p, theta=0.5, tau=1e-2)
    m2, li2, dq2, mv2 = oracle.move_sync(g, tau=1e-2)
    assert np.array_equal(m, m2)
    assert li == li2 + 1 and dq[0] == 0.0 and np.array_equal(dq[1:], dq2)
    assert cnt["pruned"] == int(np.count_nonzero(np.diff(g.offsets))) and cnt["confirm_sweeps"] == 1


def test_gate_that_prunes_nothing_follows_the_plain_trajectory():
    g = gi.dcsbm_small(6000, 3)
    p = np.zeros(P, np.float32)
    p[B3] = 30.0
    m, li, dq, mv, cnt = oracle.move_sync_gated(g, p, theta=0.5, tau=1e-2)
    m2, li2, dq2, mv2 = oracle.move_sync(g, tau=1e-2)
    assert cnt["pruned"] == 0 and cnt["confirm_sweeps"] == 1
    assert li >= li2 and np.array_equal(dq[:li2], dq2) and np.array_equal(mv[:li2], mv2)
    if li == li2:                       # the confirming sweep moved nothing
        assert np.array_equal(m, m2)


def test_traces_of_a_plain_phase():
    """Rate 1: one row per scan; labels sum to the movers of each sweep; the
    first sweep's features describe never-scanned singletons."""
    g = gi.dcsbm_small(3000, 4)
    tr = oracle.Trace(200_000, seed=5, rate=1.0)
    m, li, dq, mv, cnt = oracle.move_sync_gated(g, None, tau=1e-2, trace=tr, pass_index=3)
    x, y, v, meta = tr.arrays()
    assert tr.rows == tr.seen == cnt["scanned_vertices"]
    sweeps = meta % 256
    assert np.all(meta // 256 == 3)
    for s in range(li):
        assert int(y[sweeps == s].sum()) == int(mv[s])
    first = sweeps == 0
    assert np.all(x[first][:, 6] == 0) and np.all(x[first][:, 4] == 0) and np.all(x[first][:, 3] == 0.375)
    # vertices of the first sub-round see the initial singletons: K_i / Sigma_i = 1
    sub0 = np.array([((int(i) * 0x9E3779B97F4A7C15) % 2 ** 64) >> 61 == 0 for i in v]) & first
    deg = np.diff(g.offsets)[v[sub0]]
    assert sub0.sum() > 100 and np.all(x[sub0][:, 5] == np.where(deg > 0, 1.0, 0.0))
    later = sweeps > 0
    assert np.any(x[later][:, 6] == 1) and np.any(x[later][:, 6] == 0.5)
    # D_i: a vertex re-marked in a later sweep had a neighbour move, so D_i > 0
    assert np.all(x[later][:, 7] > 0)
    # sampling: at rate 1/4 the kept rows are those the predicate selects
    tr2 = oracle.Trace(200_000, seed=5, rate=0.25)
    oracle.move_sync_gated(g, None, tau=1e-2, trace=tr2, pass_index=3)
    thr = int(0.25 * 2 ** 64)
    x2, y2, v2, meta2 = tr2.arrays()
    keep = np.array([oracle.trace_keep(5, 3, int(s), int(i), thr) for s, i in zip(sweeps, v)])
    assert tr2.rows == int(keep.sum())
    assert np.array_equal(v2, v[keep]) and np.array_equal(y2, y[keep]) and np.array_equal(x2, x[keep])
