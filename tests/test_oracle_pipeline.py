"""Pins of the oracle's solver and SS-FNO/NAF pipeline."""
import numpy as np
import pytest

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


# ---------------------------------------------------------------------------
# The densities of the SS-FNO step pinned to their definitions in the determinant spaces of the
# intermediate-state oracle (tier 0): one-particle densities <Psi| c+_p c_q |Psi> of explicit
# (N+1)- and N-electron vectors, built from creation and annihilation operators.
# ---------------------------------------------------------------------------
from oracle import adc_so  # noqa: E402
from oracle.adc_cs import z_to_x  # noqa: E402
from oracle.isr import ISR  # noqa: E402


def _tier0(o=2, v=3, X=6, seed=5, sc=0.4):
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=sc)
    return eo, ev, B, ISR(eo, ev, B), Problem(eo, ev, B)


def _density(isr, bra, ket, p, q, nelec):
    return bra @ (isr.lad.one_body(p, q, nelec) @ ket)


def _reference_det(isr):
    S = isr.lad.spaces[isr.N]
    phi0 = np.zeros(S.dim)
    phi0[S.index[(1 << isr.N) - 1]] = 1.0
    return phi0


def _state_vector(isr, o, v, vec):
    """(N+1)-electron determinant vector of the zeroth-order intermediate states with doublet coordinates
    vec = (r1, z): sum_A u_A c+_A Phi0 + sum_(A<B, I) u_ABI c+_A c+_B c_I Phi0, u = C vec (spin-orbitals)."""
    N = isr.N
    u = adc_so.doublet_embedding(o, v) @ vec
    phi0 = _reference_det(isr)
    nv = 2 * v
    out = np.zeros(isr.lad.spaces[N + 1].dim)
    for A in range(nv):
        out += u[A] * isr.lad.apply("c", N + A, N, phi0)
    cls2 = [(A, B, I) for A in range(nv) for B in range(nv) if A < B for I in range(2 * o)]
    for k, (A, B, I) in enumerate(cls2):
        if u[nv + k] != 0.0:
            w = isr.lad.apply("a", I, N, phi0)
            w = isr.lad.apply("c", N + B, N - 1, w)
            out += u[nv + k] * isr.lad.apply("c", N + A, N, w)
    return out


def _spin_averaged_vv(isr, o, v, psi, nelec):
    ra = np.array([[_density(isr, psi, psi, 2 * (o + a), 2 * (o + b), nelec) for b in range(v)] for a in range(v)])
    rb = np.array([[_density(isr, psi, psi, 2 * (o + a) + 1, 2 * (o + b) + 1, nelec) for b in range(v)]
                   for a in range(v)])
    return 0.5 * (ra + rb)


def _ea_density_swapped_beta(P, vec):
    """A plausible mistake: the beta electron's term with the index order of the alpha one."""
    r1, z = P.split(vec)
    x = z_to_x(z)
    y = x - x.transpose(0, 2, 1)
    rho = np.outer(r1, r1) + 2.0 * np.einsum("iac,ibc->ab", x, x) + np.einsum("iac,ibc->ab", y, y)
    return 0.5 * rho


def _ea_density_x_for_y(P, vec):
    """A plausible mistake: the same-spin amplitudes y replaced by x."""
    r1, z = P.split(vec)
    x = z_to_x(z)
    rho = np.outer(r1, r1) + 2.0 * np.einsum("iac,ibc->ab", x, x) + np.einsum("ica,icb->ab", x, x)
    return 0.5 * rho


@pytest.mark.parametrize("case", [(2, 3, 6, 5, 0.4), (1, 4, 5, 7, 0.6)])
def test_ea_density_is_the_determinant_density(case):
    """D^EA (eq 17 reading) = the spin-averaged virtual density of the (N+1)-electron state that the
    doublet coordinates describe on the zeroth-order intermediate states (c+_a Phi0, c+_a c+_b c_i Phi0):
    for a random state and for ADC(2) eigenvectors.  Two plausible mistakes must fail."""
    o, v = case[0], case[1]
    eo, ev, B, isr, P = _tier0(*case)
    rng = np.random.default_rng(1)
    vecs = [rng.standard_normal(P.dim())]
    w, Y = np.linalg.eigh(P.dense(2))
    vecs += [Y[:, 0], Y[:, 2]]
    for vec in vecs:
        vec = vec / np.linalg.norm(vec)
        psi = _state_vector(isr, o, v, vec)
        assert abs(psi @ psi - 1.0) < 1e-13
        ref = _spin_averaged_vv(isr, o, v, psi, isr.N + 1)
        D = ssfno.ea_density(P, vec)
        assert np.abs(D - ref).max() < 1e-14
        assert np.abs(_ea_density_swapped_beta(P, vec) - ref).max() > 1e-8
        assert np.abs(_ea_density_x_for_y(P, vec) - ref).max() > 1e-8


@pytest.mark.parametrize("case", [(2, 3, 6, 5, 0.4), (1, 4, 5, 7, 0.6), (2, 4, 7, 3, 0.3)])
def test_mp2_densities_are_the_second_order_densities(case):
    """D^MP2 (per spin, eq 17 reading), the occupied block and the singles u1 that enter the static
    self-energy = the second-order one-particle densities of the Rayleigh-Schroedinger ground state
    Psi0 = Phi0 + Psi1 + Psi2 (intermediate normalisation): vv <Psi1|c+_a c_b|Psi1>,
    oo <Psi1|c+_i c_j|Psi1> - delta_ij <Psi1|Psi1>, ov <Phi0|c+_i c_a|Psi2>."""
    o, v = case[0], case[1]
    eo, ev, B, isr, P = _tier0(*case)
    N = isr.N
    psi1, psi2 = isr.psi0[1], isr.psi0[2]
    phi0 = _reference_det(isr)
    vv = np.array([[_density(isr, psi1, psi1, 2 * (o + a), 2 * (o + b), N) for b in range(v)] for a in range(v)])
    oo = np.array([[_density(isr, psi1, psi1, 2 * i, 2 * j, N) - (i == j) * (psi1 @ psi1) for j in range(o)]
                   for i in range(o)])
    ov = np.array([[_density(isr, phi0, psi2, 2 * i, 2 * (o + a), N) for a in range(v)] for i in range(o)])
    assert np.abs(vv).max() > 1e-4 and np.abs(oo).max() > 1e-4 and np.abs(ov).max() > 1e-5
    assert np.abs(P.mp2_density_vv() - vv).max() < 1e-15
    assert np.abs(P.mp2_density_oo() - oo).max() < 1e-15
    assert np.abs(P.second_order()[3] - ov).max() < 1e-15
    # a plausible mistake: the exchange-like term with the wrong sign
    T = P.T
    wrong = np.einsum("klce,klcd->ed", 2.0 * T + T.transpose(0, 1, 3, 2), T)
    assert np.abs(wrong - vv).max() > 1e-6


def _matching_detail(o, v, X, seed, sc, thr, k, nroots=4):
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=sc)
    P0 = Problem(eo, ev, B)
    w2, Y2, _ = ssfno.solve_roots(P0, 2, nroots, 1e-10)
    Dss = P0.mp2_density_vv() + ssfno.ea_density(P0, Y2[k])
    U, en, eta, nk = ssfno.natural_orbitals(Dss, ev, thr)
    Pk = Problem(eo, en, ssfno.transform_B(B, o, U))
    w2k, Y2k, _ = ssfno.solve_roots(Pk, 2, nroots, 1e-10)
    ref = ssfno.carry_vector(Y2[k], o, v, U)
    m_full = int(np.argmax(np.abs(Y2k @ ref)))
    m_1p = int(np.argmax(np.abs(Y2k[:, :nk] @ ref[:nk])))
    r1norm = float(np.linalg.norm(Y2[k][:v]))
    return w2, w2k, m_full, m_1p, r1norm, (eo, ev, B)


def test_root_matching_follows_the_state_through_reordering():
    """Root k of a truncated basis (eq 30 needs the same state in both bases).  A mild change of basis
    moves a state's energy only slightly, so the matched truncated ADC(2) root must lie close to the
    canonical one.  (a) A 1p-dominated state that the truncation reorders (canonical root 3 becomes
    truncated root 1): the full-vector overlap rule and the 1p-overlap rule both pick it, index
    matching would not.  (b) A 2p1h satellite (|r1| ~ 0.03): the full-vector rule follows it; the
    1p-overlap rule, whose overlaps are all ~1e-3 there, picks a state 0.29 Eh away."""
    w2, w2k, m_full, m_1p, r1n, inst = _matching_detail(2, 8, 16, 5, 0.05, 1e-3, 3)
    assert r1n > 0.99 and m_full == m_1p == 1
    assert abs(w2k[m_full] - w2[3]) < 1e-3 and abs(w2k[3] - w2[3]) > 1e-3
    eo, ev, B = inst
    run = ssfno.run(eo, ev, B, 4, 1e-3, 0.0, 1e-10)
    assert abs(run["omega_adc2_fno"][3] - w2k[1]) < 1e-12
    w2, w2k, m_full, m_1p, r1n, _ = _matching_detail(2, 8, 16, 7, 0.1, 1e-4, 1)
    assert r1n < 0.05 and m_full == 1 and m_1p != m_full
    assert abs(w2k[m_full] - w2[1]) < 1e-3 < abs(w2k[m_1p] - w2[1])


@pytest.mark.parametrize("case", [(2, 3, 6, 5, 0.4), (1, 4, 5, 7, 0.6)])
def test_sm_adc_against_intermediate_states(case):
    """Scaled-matrix ADC (the equation after eq 5; reading M_ADC(2) + x (M_ADC(3) - M_ADC(2))): the
    oracle's matrix equals C^T [M2 + x (M3 - M2)] C with M2, M3 the order-truncated intermediate-state
    matrices of tier 0 (x = 0 gives ADC(2), x = 1 ADC(3), as the paper states), and the part x scales is
    exactly M11 at third order, the coupling at second order and the 2p1h block at first order."""
    o, v = case[0], case[1]
    eo, ev, B, isr, P = _tier0(*case)
    C = adc_so.doublet_embedding(o, v)
    M2, M3 = isr.adc_matrix(2), isr.adc_matrix(3)
    n1 = 2 * v
    third = np.zeros_like(M2)
    third[:n1, :n1] = isr.M[3][:n1, :n1]
    third[:n1, n1:] = isr.M[2][:n1, n1:]
    third[n1:, :n1] = isr.M[2][n1:, :n1]
    third[n1:, n1:] = isr.M[1][n1:, n1:]
    assert np.abs((M3 - M2) - third).max() < 1e-14
    for x in (0.0, 0.5, 0.3, 1.0):
        ref = C.T @ (M2 + x * third) @ C
        assert np.abs(P.dense_sm(x).T - ref).max() < 1e-12
        assert np.abs(P.diagonal_sm(x) - np.diag(ref)).max() < 1e-12
    assert np.abs(P.dense_sm(0.0) - P.dense(2)).max() < 1e-13
    assert np.abs(P.dense_sm(1.0) - P.dense(3)).max() < 1e-13


def test_mp2_fno_and_share_of_virtuals():
    """Ground-state MP2-FNO: every root in the one basis of D^MP2; the percentage-of-virtuals truncation
    keeps ceil(frac v) orbitals; nothing truncated reproduces canonical ADC(3); the shared basis equals the
    state-specific pipeline run on D^MP2 alone (here: same kept counts for all roots)."""
    eo, ev, B = synth.make_instance(3, 10, 24, 8, 0.3)
    can = ssfno.run(eo, ev, B, 3, 0.0, 0.0, 1e-9)["roots"]
    r = ssfno.run(eo, ev, B, 3, 1e-300, 0.0, 1e-9, fno_mode="mp2")
    assert r["nvir_kept"] == [10] * 3 and np.abs(r["roots"] - can).max() < 1e-10
    r = ssfno.run(eo, ev, B, 3, 0.0, 0.0, 1e-9, keep_frac=1.0)
    assert r["nvir_kept"] == [10] * 3 and np.abs(r["roots"] - can).max() < 1e-10
    r = ssfno.run(eo, ev, B, 3, 0.0, 0.0, 1e-9, fno_mode="mp2", keep_frac=0.55)
    assert r["nvir_kept"] == [6] * 3
    U, e, eta, k = ssfno.natural_orbitals(Problem(eo, ev, B).mp2_density_vv(), ev, 0.0, 6)
    assert k == 6 and np.all(eta[:6] >= eta[6:].max())
    s = ssfno.run(eo, ev, B, 3, 0.0, 0.0, 1e-9, keep_frac=0.55)
    assert s["nvir_kept"] == [6] * 3
    # the state-specific densities pick other orbitals than D^MP2 alone
    assert np.abs(np.array(s["roots"]) - np.array(r["roots"])).max() > 1e-8


def _tier0_transition_series(isr):
    """Order coefficients of f_Ap = <Psi~_A| c+_p |Psi0> (eq 8) from the tier-0 intermediate states, with
    Psi0 normalised (the series is kept in intermediate normalisation); p runs over spin-orbitals."""
    from oracle.isr import ORDER
    N, psi = isr.N, isr.psi0
    S = np.array([sum(psi[k] @ psi[n - k] for k in range(n + 1)) for n in range(ORDER + 1)])
    inv = np.zeros(ORDER + 1)
    inv[0], inv[2], inv[3] = 1.0, -0.5 * S[2], -0.5 * S[3]
    psin = np.array([sum(inv[k] * psi[n - k] for k in range(n + 1)) for n in range(ORDER + 1)])
    norb = isr.lad.spaces[N].norb
    f = np.zeros((ORDER + 1, isr.Y.shape[1], norb))
    for n in range(ORDER + 1):
        for k in range(n + 1):
            cp = np.stack([isr.lad.apply("c", p, N, psin[n - k]) for p in range(norb)])
            f[n] += isr.Y[k] @ cp.T
    return f


@pytest.mark.parametrize("case", [(2, 3, 6, 5, 0.4), (1, 4, 5, 7, 0.6), (2, 4, 7, 3, 0.3)])
def test_transition_amplitudes_against_intermediate_states(case):
    """f (eq 8) of the oracle = the tier-0 series of <Psi~_A| c+_p alpha |Psi0> in doublet coordinates,
    through second order in the 1p rows and first order in the 2p1h rows; the first-order 1p rows and the
    first-order 2p1h rows of virtual p vanish identically.  Sum rule of the 1p rows' virtual columns and the
    2p1h rows' occupied columns: f^T f = 1 - (second-order occupation) through second order, i.e.
    delta - D^MP2 (vv) and -D^MP2_oo (oo)."""
    o, v = case[0], case[1]
    eo, ev, B, isr, P = _tier0(*case)
    C = adc_so.doublet_embedding(o, v)
    fs = _tier0_transition_series(isr)
    fz = [C.T @ fs[n][:, 0::2] for n in range(fs.shape[0])]  # alpha spin-orbitals -> spatial columns
    f = P.transition_amplitudes()
    ref = np.zeros_like(f)
    ref[:v] = fz[0][:v] + fz[1][:v] + fz[2][:v]
    ref[v:] = fz[0][v:] + fz[1][v:]
    assert np.abs(f - ref).max() < 1e-14
    assert np.abs(fz[1][:v]).max() < 1e-15 and np.abs(fz[1][v:, o:]).max() < 1e-15
    assert np.abs(fz[2][:v, :o]).max() > 1e-5  # the second-order singles do enter
    ftf = f.T @ f
    D = P.mp2_density_vv()
    u1 = P.second_order()[3]
    # virtual columns: (1 - D/2)^2 = 1 - D through second order
    assert np.abs(ftf[o:, o:] - (np.eye(v) - D + 0.25 * D @ D)).max() < 1e-14
    # occupied columns: the 2p1h rows' norm is the second-order hole occupation -D_oo (an identity of the
    # z transform that ties f's normalisation to the pinned occupied density), plus the singles' square
    assert np.abs(ftf[:o, :o] - u1 @ u1.T + P.mp2_density_oo()).max() < 1e-14


def test_spectral_amplitudes_of_roots():
    """x = Y^T f (eq 7) for the lowest ADC(3) roots; a 1p-dominated root has pole strength near 1 and a
    2p1h satellite a small one; x equals the tier-0 amplitudes of the same eigenvectors."""
    o, v = 2, 3
    eo, ev, B, isr, P = _tier0(o, v, 6, 5, 0.4)
    w, Y = np.linalg.eigh(P.dense(3))
    x = P.spectral_amplitudes(Y.T)
    ps = np.sum(x * x, axis=1)
    r1 = np.sum(Y[:v] ** 2, axis=0)
    assert ps[np.argmax(r1)] > 0.9 and ps[np.argmin(r1)] < 0.1
    C = adc_so.doublet_embedding(o, v)
    fs = _tier0_transition_series(isr)
    f0 = C.T @ (fs[0] + fs[1] + fs[2])[:, 0::2]
    f0[v:] = (C.T @ (fs[0] + fs[1])[:, 0::2])[v:]
    assert np.abs(x - Y.T @ f0).max() < 1e-14
