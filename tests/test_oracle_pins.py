"""Pins of the FP64 oracle against things other than itself.

* tier 0 (numerical ISR) against brute-force FCI: ADC(2) errors shrink as lam^3,
  ADC(3) errors as lam^4 (eq 5 truncation), also for an exactly degenerate
  virtual pair; its second-order energy equals the textbook MP2 energy; the
  lam^2 coefficient of a 1p root equals the closed-form second-order EA.
* tier 1 (closed-form spin-orbital M) against tier 0, element by element.
* tier 2 (closed-shell DF sigma in doublet coordinates) against C^T M_so C.
"""
import numpy as np
import pytest

import synth
from oracle import adc_so
from oracle.adc_cs import Problem
from oracle.isr import ISR, spin_orbital_tensors

CASES = [(2, 3, 6, 5, 0.4), (1, 4, 5, 7, 0.6), (2, 4, 7, 3, 0.3)]


def _inst(o, v, X, seed, sc):
    return synth.make_instance(o, v, X, seed, scale=sc)


@pytest.fixture(scope="module")
def isr_cases():
    return [(c, _inst(*c), ISR(*_inst(*c))) for c in CASES]


def test_isr_hermitian_each_order(isr_cases):
    for _, _, isr in isr_cases:
        for k in range(4):
            assert np.abs(isr.M[k] - isr.M[k].T).max() < 1e-13


def _main_state_errors(isr, ev, lam, level):
    ex = isr.fci_ea(lam)
    w = np.linalg.eigvalsh(isr.adc_matrix(level, lam))
    errs = []
    for e in ev:
        tgt = w[np.argmin(abs(w - e))]
        errs.append(tgt - ex[np.argmin(abs(ex - tgt))])
    return np.array(errs)


@pytest.mark.parametrize("degenerate", [False, True])
def test_isr_order_consistency_vs_fci(degenerate):
    eo, ev, B = _inst(2, 3, 6, 5, 0.4)
    if degenerate:
        ev = ev.copy()
        ev[2] = ev[1]  # exactly degenerate virtual pair
    isr = ISR(eo, ev, B)
    for level, power in ((2, 3), (3, 4)):
        e1 = _main_state_errors(isr, ev, 0.05, level)
        e2 = _main_state_errors(isr, ev, 0.025, level)
        ratio = np.abs(e1 / e2)
        assert np.all(np.abs(ratio / 2 ** power - 1) < 0.08), (level, ratio)


def test_isr_second_order_energy_is_mp2():
    eo, ev, B = _inst(2, 3, 6, 5, 0.4)
    isr = ISR(eo, ev, B)
    eps, g = spin_orbital_tensors(eo, ev, B)
    no = 2 * eo.size
    o, v = slice(0, no), slice(no, None)
    D = eps[o][:, None, None, None] + eps[o][None, :, None, None] - eps[v][None, None, :, None] - eps[v][None, None, None, :]
    e2 = 0.25 * np.sum(g[o, o, v, v] ** 2 / D)
    assert abs(isr.E0[2] - e2) < 1e-13
    assert abs(Problem(eo, ev, B).mp2_energy() - e2) < 1e-12


def test_isr_second_order_ea_closed_form():
    """lam^2 coefficient of a non-degenerate 1p root = RSPT second-order EA."""
    eo, ev, B = _inst(2, 3, 6, 5, 0.4)
    isr = ISR(eo, ev, B)
    eps, g = spin_orbital_tensors(eo, ev, B)
    no = 2 * eo.size
    occ, vir = range(no), range(no, eps.size)
    A = no  # alpha spin-orbital of the lowest virtual
    e2 = 0.0
    for i in occ:
        for b in vir:
            for c in vir:
                if b < c:
                    e2 += g[b, c, A, i] ** 2 / (eps[A] + eps[i] - eps[b] - eps[c])
    for i in occ:
        for j in occ:
            for c in vir:
                e2 -= 0.5 * g[A, c, i, j] ** 2 / (eps[i] + eps[j] - eps[A] - eps[c])
    for lam in (1e-3,):
        w = np.linalg.eigvalsh(isr.adc_matrix(2, lam))
        w0 = w[np.argmin(abs(w - ev[0]))]
        assert abs((w0 - ev[0]) / lam ** 2 - e2) < 1e-3 * abs(e2) + 1e-9


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("level", [2, 3])
def test_closed_form_spin_orbital_matches_isr(case, level):
    eo, ev, B = _inst(*case)
    Mi = ISR(eo, ev, B).adc_matrix(level)
    Mc = adc_so.dense_matrix(eo, ev, B, level)
    assert np.abs(Mi - Mc).max() < 1e-13


@pytest.mark.parametrize("case", CASES + [(3, 3, 5, 11, 0.5)])
@pytest.mark.parametrize("level", [2, 3])
def test_closed_shell_sigma_matches_spin_orbital(case, level):
    o, v = case[0], case[1]
    eo, ev, B = _inst(*case)
    C = adc_so.doublet_embedding(o, v)
    assert np.abs(C.T @ C - np.eye(C.shape[1])).max() < 1e-14
    Mso = adc_so.dense_matrix(eo, ev, B, level)
    # the doublet space is invariant under M
    assert np.abs(Mso @ C - C @ (C.T @ Mso @ C)).max() < 1e-12
    P = Problem(eo, ev, B)
    Md = P.dense(level).T
    assert np.abs(Md - C.T @ Mso @ C).max() < 1e-12
    assert np.abs(Md - Md.T).max() < 1e-12
    assert np.abs(np.diag(Md) - P.diagonal(level)).max() < 1e-12


def test_df_integrals():
    eo, ev, B = _inst(3, 5, 9, 2, 1.0)
    g = np.einsum("Qpq,Qrs->pqrs", B, B)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.abs(g - g.transpose(perm)).max() < 1e-14
    P = Problem(eo, ev, B)
    o = 3
    assert np.abs(P.ovov - g[:o, o:, :o, o:]).max() < 1e-13
    assert np.abs(P.oovv - g[:o, :o, o:, o:]).max() < 1e-13
    x = np.random.default_rng(0).standard_normal((2, o, 5, 5))
    ref = np.einsum("acbd,nicd->niab", g[o:, o:, o:, o:], x)
    assert np.abs(P.vvvv_apply(x) - ref).max() < 1e-12
    big = np.random.default_rng(1).standard_normal((200, 5, 5))
    ref = np.einsum("acbd,ncd->nab", g[o:, o:, o:, o:], big)
    assert np.abs(P.vvvv_apply(big) - ref).max() < 1e-11


def test_mp2_density_traces():
    eo, ev, B = _inst(4, 12, 30, 4, 0.3)
    P = Problem(eo, ev, B)
    assert abs(np.trace(P.mp2_density_vv()) + np.trace(P.mp2_density_oo())) < 1e-12
    D = P.mp2_density_vv()
    assert np.abs(D - D.T).max() < 1e-14


def test_ladder_rows_match_full_ladder():
    """The oracle's row sampler of the ladder equals the explicit four-index contraction."""
    from oracle.adc_cs import ladder_rows
    eo, ev, B = _inst(2, 7, 9, 4, 1.0)
    g = np.einsum("Qpq,Qrs->pqrs", B, B)[2:, 2:, 2:, 2:]
    amp = np.random.default_rng(2).standard_normal((7, 7))
    full = np.einsum("acbd,cd->ab", g, amp)
    rows = [0, 3, 6]
    assert np.abs(ladder_rows(B[:, 2:, 2:], amp, rows) - full[rows]).max() < 1e-12 * np.abs(full).max()
