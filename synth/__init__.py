"""Seeded synthetic inputs for the DF-EA-ADC problem.

This module only draws numbers: closed-shell orbital energies and a
three-index density-fitting factor B^Q_pq (the J^Q_pq of the DF
factorisation (pq|rs) = sum_Q J^Q_pq J^Q_rs, Sec. "Density Fitting (DF)
Approximation", eqs 25-26).  It holds none of the method's arithmetic and is
the only code shared by the FP64 oracle and the GPU path.

Recipe (fixed draw order, so a seed names one instance):
  rng      = numpy.random.default_rng(seed)
  eps_occ  = sort(rng.uniform(-1.5, -0.3, nocc))        [Eh]
  eps_vir  = sort(rng.uniform(0.05, 3.0, nvir))         [Eh]
  G        = rng.standard_normal((naux, n, n)),  n = nocc + nvir
  B[Q,p,q] = B[Q,q,p] = scale * 0.3 * exp(-Q/20) * G[Q, min(p,q), max(p,q)]
MO order is occupied first, then virtual.  ``scale`` = 1 is the literal
workload; a smaller ``scale`` gives a weakly correlated variant in which the
natural-orbital truncation actually removes virtuals.
"""
import numpy as np

__all__ = ["make_instance", "preset", "batch_shapes", "PRESETS", "mlp_init", "mlp_features_draw"]


def make_instance(nocc, nvir, naux, seed, scale=1.0, rng=None):
    """Return (eps_occ[nocc], eps_vir[nvir], B[naux, n, n]) as float64 arrays."""
    if rng is None:
        rng = np.random.default_rng(seed)
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, nocc))
    eps_vir = np.sort(rng.uniform(0.05, 3.0, nvir))
    n = nocc + nvir
    G = rng.standard_normal((naux, n, n))
    up = np.triu(G)
    B = up + np.transpose(np.triu(G, 1), (0, 2, 1))
    del G, up
    B *= (scale * 0.3 * np.exp(-np.arange(naux) / 20.0))[:, None, None]
    return eps_occ, eps_vir, np.ascontiguousarray(B)


def batch_shapes(seed):
    """Shape of one instance of the ragged batch: nocc~U{5..30}, nvir~U{50..300}, naux=3*nvir.

    The same generator then continues with make_instance's draws."""
    rng = np.random.default_rng(seed)
    nocc = int(rng.integers(5, 31))
    nvir = int(rng.integers(50, 301))
    return rng, nocc, nvir, 3 * nvir


def batch_instance(seed, scale=1.0):
    rng, o, v, x = batch_shapes(seed)
    return make_instance(o, v, x, seed, scale=scale, rng=rng)


# Named workloads: (nocc, nvir, naux, seed, nroots, fno_thresh, naf_thresh, conv)
PRESETS = {
    "tiny-dense": dict(nocc=4, nvir=20, naux=60, seed=0, nroots=3,
                       fno_thresh=0.0, naf_thresh=0.0, conv=1e-8),
    "ssfno-o20v200x600": dict(nocc=20, nvir=200, naux=600, seed=1, nroots=5,
                              fno_thresh=10.0 ** -4.5, naf_thresh=1e-2, conv=1e-6),
    "mixed-o40v600x1800": dict(nocc=40, nvir=600, naux=1800, seed=2, nroots=5,
                               fno_thresh=0.0, naf_thresh=0.0, conv=1e-6),
    "learned-o30v400x1200": dict(nocc=30, nvir=400, naux=1200, seed=240, nroots=5,
                                 fno_thresh=0.0, naf_thresh=0.0, conv=1e-6),
}


def preset(name, scale=1.0):
    p = dict(PRESETS[name])
    eo, ev, B = make_instance(p["nocc"], p["nvir"], p["naux"], p["seed"], scale=scale)
    return p, eo, ev, B


# Learned-preconditioner network: 6 -> 256 -> 256 -> 1, flat float32 layout
# W1[6][256], b1[256], W2[256][256], b2[256], W3[256], b3[1].
MLP_SIZES = (6 * 256, 256, 256 * 256, 256, 256, 1)


def mlp_init(seed, head_scale=0.0):
    """Initial weights: W1 ~ N(0, 1/6), W2 ~ N(0, 1/256), zero biases, W3 ~ head_scale * N(0, 1/256), b3 = 0.

    head_scale = 0 makes the initial network output zero everywhere."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal(6 * 256) / np.sqrt(6.0)
    W2 = rng.standard_normal(256 * 256) / 16.0
    W3 = head_scale * rng.standard_normal(256) / 16.0
    w = np.concatenate([W1, np.zeros(256), W2, np.zeros(256), W3, np.zeros(1)])
    return w.astype(np.float32)


def mlp_features_draw(n_groups, group, seed):
    """Random (features[G*S, 6], a0[G*S], target[G*S]) of feature-like magnitudes for kernel checks."""
    rng = np.random.default_rng(seed)
    n = n_groups * group
    F = np.empty((n, 6))
    F[:, 0] = rng.uniform(0.0, 4.0, n)
    F[:, 1] = rng.standard_normal(n)
    F[:, 2] = (rng.uniform(size=n) < 0.1).astype(np.float64)
    F[:, 3] = rng.uniform(0.05, 3.0, n)
    F[:, 4] = rng.uniform(0.05, 3.0, n) * (1 - F[:, 2])
    F[:, 5] = rng.uniform(-1.5, -0.3, n) * (1 - F[:, 2])
    a0 = rng.standard_normal(n) * 1e-3
    d = a0 * (1.0 + 0.3 * rng.standard_normal(n)) + 1e-4 * rng.standard_normal(n)
    return F, a0, d
