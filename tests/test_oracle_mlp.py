"""Pins of the FP64 learned-preconditioner reference (oracle/mlp_ref.py)."""
import numpy as np
import pytest

from oracle import mlp_ref
import synth


def _data(G=3, S=17, seed=5):
    F, a0, d = synth.mlp_features_draw(G, S, seed)
    w = synth.mlp_init(seed, head_scale=1.0).astype(np.float64)
    w[mlp_ref.NF * mlp_ref.H:mlp_ref.NF * mlp_ref.H + mlp_ref.H] = 0.1  # nonzero b1
    return w, F, a0, d, S


def test_nparam_layout():
    assert mlp_ref.NPARAM == 6 * 256 + 256 + 256 * 256 + 256 + 256 + 1 == sum(synth.MLP_SIZES)


def test_gelu_known_values():
    # tanh-form GELU: 0 at 0, odd part z/2 tanh(.), -> z for large z, -> 0 for very negative z
    assert mlp_ref.gelu(np.array([0.0]))[0] == 0.0
    z = np.array([1.0])
    expect = 0.5 * (1.0 + np.tanh(np.sqrt(2 / np.pi) * (1.0 + 0.044715)))
    assert abs(mlp_ref.gelu(z)[0] - expect) < 1e-15
    assert abs(mlp_ref.gelu(np.array([30.0]))[0] - 30.0) < 1e-12
    assert abs(mlp_ref.gelu(np.array([-30.0]))[0]) < 1e-12


def test_gelu_grad_central_difference():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp_ref.gelu(z + h) - mlp_ref.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp_ref.gelu_grad(z))) < 1e-8


def test_zero_head_is_jacobi():
    # W3 = b3 = 0: u = 0, so the step equals the Jacobi step and the loss is 1 - cos^2(a0, d)
    F, a0, d = synth.mlp_features_draw(2, 10, 1)
    w = synth.mlp_init(1).astype(np.float64)
    u, _ = mlp_ref.forward(w, F)
    assert np.all(u == 0.0)
    L = mlp_ref.loss(w, F, a0, d, 10)
    A, Dd = a0.reshape(2, 10), d.reshape(2, 10)
    c2 = [(A[g] @ Dd[g]) ** 2 / ((A[g] @ A[g]) * (Dd[g] @ Dd[g])) for g in range(2)]
    assert abs(L - np.mean([1 - c for c in c2])) < 1e-15


def test_loss_invariances():
    # loss of a group is invariant to scaling a0 or d and zero when a is parallel to d
    w, F, a0, d, S = _data()
    L = mlp_ref.loss(w, F, a0, d, S)
    assert abs(mlp_ref.loss(w, F, 3.0 * a0, -2.0 * d, S) - L) < 1e-13
    u, _ = mlp_ref.forward(w, F)
    a = a0 * (1 + u)
    assert abs(mlp_ref.loss(w, F, a0, 5.0 * a, S)) < 1e-13
    assert 0.0 <= L <= 1.0


def test_gradient_central_difference():
    w, F, a0, d, S = _data()
    g = mlp_ref.grad(w, F, a0, d, S)
    rng = np.random.default_rng(0)
    # every parameter block, several entries each
    offs = np.cumsum([0] + list(synth.MLP_SIZES))
    picks = []
    for b in range(6):
        n = offs[b + 1] - offs[b]
        picks += list(offs[b] + rng.choice(n, size=min(n, 6), replace=False))
    h = 1e-5
    for p in picks:
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd = (mlp_ref.loss(wp, F, a0, d, S) - mlp_ref.loss(wm, F, a0, d, S)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-7 + 1e-5 * abs(g[p]), (p, fd, g[p])


def test_gradient_directional_derivative():
    w, F, a0, d, S = _data(G=4, S=9, seed=8)
    g = mlp_ref.grad(w, F, a0, d, S)
    v = np.random.default_rng(1).standard_normal(w.size)
    h = 1e-6
    fd = (mlp_ref.loss(w + h * v, F, a0, d, S) - mlp_ref.loss(w - h * v, F, a0, d, S)) / (2 * h)
    assert abs(fd - g @ v) < 1e-6 * max(1.0, abs(g @ v))


def test_features_tiny():
    # o=1, v=2: element order [1p a=0, 1p a=1, (i0,a0,b0), (i0,a0,b1), (i0,a1,b0), (i0,a1,b1)]
    eo, ev = np.array([-0.5]), np.array([0.25, 1.5])
    D = np.array([0.3, 1.6, 1.0, 2.2, 2.3, 3.4])
    r = np.array([1.0, -1.0, 2.0, 0.0, 0.0, -2.0])
    F = mlp_ref.features(r, 0.2, D, eo, ev, 1, 2)
    rms = np.sqrt(10.0 / 6.0)
    assert np.allclose(F[:, 0], (D - 0.2) / 1.2)
    assert np.allclose(F[:, 1], r / rms)
    assert F[:, 2].tolist() == [1, 1, 0, 0, 0, 0]
    assert F[:, 3].tolist() == [0.25, 1.5, 0.25, 0.25, 1.5, 1.5]
    assert F[:, 4].tolist() == [0, 0, 0.25, 1.5, 0.25, 1.5]
    assert F[:, 5].tolist() == [0, 0, -0.5, -0.5, -0.5, -0.5]
