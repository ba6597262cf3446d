"""Pins of the oracle's solver and SS-FNO/NAF pipeline."""
import numpy as np

import synth
from oracle import ssfno
from oracle.adc_cs import Problem
from oracle.davidson import davidson


def test_davidson_equals_eigh_tiny_dense():
    """Workload o=4, v=20, X=60, seed 0: the 1620-dimensional ADC(3) matrix."""
    eo, ev, B = synth.make_instance(4, 20, 60, 0)
    P = Problem(eo, ev, B)
    assert P.dim() == 1620
    M = P.dense(3)
    w = np.linalg.eigvalsh(0.5 * (M + M.T))
    wd, X, rn, it, ok = davidson(lambda V: P.sigma(V, 3), P.diagonal(3), 3, conv=1e-8)
    assert ok
    assert np.abs(wd - w[:3]).max() < 1e-10
    # Ritz vectors are eigenvectors
    assert np.abs(P.sigma(X, 3) - wd[:, None] * X).max() < 1e-7


def test_untruncated_ssfno_is_canonical_adc3():
    eo, ev, B = synth.make_instance(3, 10, 24, 8, 0.5)
    can = ssfno.run(eo, ev, B, 3, 0.0, 0.0, 1e-9)["roots"]
    r = ssfno.run(eo, ev, B, 3, 1e-300, 1e-300, 1e-9)
    assert r["nvir_kept"] == [10] * 3 and r["naux_kept"] == [24] * 3
    assert np.abs(r["roots"] - can).max() < 1e-10
    assert np.abs(r["omega_adc2_can"] - r["omega_adc2_fno"]).max() < 1e-10


def test_naf_eigenvalues_are_singular_values_squared():
    eo, ev, B = synth.make_instance(2, 6, 15, 3)
    Bn, w, k = ssfno.naf(B, 2, 0.0)
    J = B[:, 2:, 2:].reshape(15, -1)
    s = np.linalg.svd(J, compute_uv=False)
    assert np.abs(np.sort(w)[::-1][:len(s)] - s ** 2).max() < 1e-12 * s[0] ** 2
    # no truncation: every integral unchanged
    g0 = np.einsum("Qpq,Qrs->pqrs", B, B)
    g1 = np.einsum("Qpq,Qrs->pqrs", Bn, Bn)
    assert np.abs(g0 - g1).max() < 1e-12


def test_natural_orbitals_untruncated_recanonicalise_to_canonical():
    eo, ev, B = synth.make_instance(3, 8, 20, 9, 0.2)
    P = Problem(eo, ev, B)
    U, e_new, eta, k = ssfno.natural_orbitals(P.mp2_density_vv(), ev, 0.0)
    assert k == 8
    assert np.abs(e_new - ev).max() < 1e-12
    assert np.abs(np.abs(U) - np.eye(8)).max() < 1e-12


def test_ea_density_trace_invariant():
    eo, ev, B = synth.make_instance(3, 7, 20, 6, 0.5)
    P = Problem(eo, ev, B)
    rng = np.random.default_rng(3)
    vec = rng.standard_normal(P.dim())
    vec /= np.linalg.norm(vec)
    D = ssfno.ea_density(P, vec)
    r1, z = P.split(vec)
    # spin-summed trace = |r1|^2 + 2 |2p1h|^2
    assert abs(2 * np.trace(D) - (r1 @ r1 + 2 * np.sum(z * z))) < 1e-12
