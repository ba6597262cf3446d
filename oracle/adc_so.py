"""Tier-1 oracle: explicit spin-orbital EA-ADC(2)/ADC(3) secular matrix.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module.

The paper's programmable sigma expressions live in its (unavailable)
supplementary material (Sec. "Algebraic Diagrammatic Construction (ADC)
Theory").  The closed forms below were derived for this project from the ISR
definition (eqs 1-5): the EA intermediate-state matrix through third order was
expanded with the Wick theorem as the one- and two-body parts of the
similarity-transformed Hamiltonian exp(-A) H exp(A), A = sigma - sigma^+, with
sigma the first- and second-order Moller-Plesset excitation operators.  Every
block is pinned elementwise to the numerical ISR of ``oracle.isr`` (tests).

Notation (spin-orbitals, real):  g[p,q,r,s] = <pq||rs>;
t[i,j,a,b]  = <ab||ij> / D_ij^ab,  D_ij^ab = e_i + e_j - e_a - e_b   (first order)
y[i,j,a,b]  = D * u  (second-order doubles residual),  u1[i,a] second-order singles.

Blocks (basis: 1p |a> = c+_a Phi0;  2p1h |abi> = c+_a c+_b c_i Phi0, a<b):
  M11 = e_a d_ab + M11^(2) + M11^(3)
  U   = <ai||bc> + U^(2)               (1p-2p1h coupling)
  K   = (e_a + e_b - e_i) + K^(1)     (2p1h-2p1h)
ADC(2) keeps M11 through 2nd order, U through 1st, K through 0th.
"""
import numpy as np

from .isr import spin_orbital_tensors

ein = lambda s, *a: np.einsum(s, *a, optimize=True)  # noqa: E731


def amplitudes(eps_so, g, no):
    """First-order t, second-order doubles residual y and amplitude u, singles u1."""
    o, v = slice(0, no), slice(no, None)
    eo, ev = eps_so[o], eps_so[v]
    D2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    D1 = eo[:, None] - ev[None, :]
    goovv = g[o, o, v, v]             # <ij||ab>
    t = goovv / D2                    # t[i,j,a,b] = <ab||ij>/D (real integrals)
    gvvvv, goooo, gvoov = g[v, v, v, v], g[o, o, o, o], g[v, o, o, v]
    # second-order doubles residual: ladder + hole ladder + four ring terms
    y = 0.5 * ein("ijcd,abcd->ijab", t, gvvvv)
    y += 0.5 * ein("klab,klij->ijab", t, goooo)
    ring = ein("ikac,bkjc->ijab", t, gvoov)       # t_ik^ac <bk||jc>
    y += ring - ring.transpose(1, 0, 2, 3) - ring.transpose(0, 1, 3, 2) + ring.transpose(1, 0, 3, 2)
    u = y / D2
    # second-order singles
    y1 = 0.5 * ein("ikcd,akcd->ia", t, g[v, o, v, v]) - 0.5 * ein("klac,klic->ia", t, g[o, o, o, v])
    u1 = y1 / D1
    return t, y, u, u1


def blocks(eps_occ, eps_vir, B, level):
    """Dense M11 [nv,nv], U[nv, nv, nv, no] (antisymmetric in the middle pair) and the
    K^(1) tensor K1[a,b,i,c,d,j] (level 3 only), all in spin-orbitals."""
    eps_so, g = spin_orbital_tensors(eps_occ, eps_vir, B)
    no = 2 * eps_occ.size
    o, v = slice(0, no), slice(no, None)
    ev = eps_so[v]
    t, y, u, u1 = amplitudes(eps_so, g, no)
    gvvoo, goovv = g[v, v, o, o], g[o, o, v, v]
    # second order (the average-of-denominators form)
    m2 = -0.25 * ein("klac,klbc->ab", t, goovv) - 0.25 * ein("klbc,ackl->ab", t, gvvoo)
    M11 = np.diag(ev) + m2
    # U^(1)[a,b,c,i] = <ai||bc>
    U = g[v, o, v, v].transpose(0, 2, 3, 1).copy()
    K1 = None
    if level >= 3:
        # third order: static self-energy with the second-order density ...
        m3 = -0.5 * ein("klcd,kmcd,ambl->ab", t, t, g[v, o, v, o])
        m3 += 0.5 * ein("klcd,klce,aebd->ab", t, t, g[v, v, v, v])
        m3 += ein("kc,acbk->ab", u1, g[v, v, v, o]) + ein("kc,akbc->ab", u1, g[v, o, v, v])
        # ... the second-order form with second-order amplitudes ...
        m3 += -0.25 * ein("klac,klbc->ab", u, goovv) - 0.25 * ein("klbc,ackl->ab", u, gvvoo)
        m3 += 0.25 * ein("klac,klbc->ab", t, y) + 0.25 * ein("klbc,klac->ab", t, y)
        # ... and the remaining products of two first-order amplitudes
        m3 += -ein("klcd,kmac,dmbl->ab", t, t, g[v, o, v, o])
        m3 += -0.25 * ein("klcd,klae,cdbe->ab", t, t, g[v, v, v, v])
        m3 += -ein("klcd,kmbc,aldm->ab", t, t, g[v, o, v, o])
        m3 += -0.25 * ein("klcd,klbe,aecd->ab", t, t, g[v, v, v, v])
        m3 += -0.25 * ein("klac,mnbc,klmn->ab", t, t, g[o, o, o, o])
        m3 += ein("klac,kmbd,dlcm->ab", t, t, g[v, o, v, o])
        M11 = M11 + m3
        # U^(2)[a,b,c,i]
        U += 0.5 * ein("klbc,aikl->abci", t, g[v, o, o, o])
        U += -ein("ikbd,adck->abci", t, g[v, v, v, o])
        U += ein("ikcd,adbk->abci", t, g[v, v, v, o])
        # K^(1)[a,b,i,c,d,j] = d_ij <ab||cd> - d_ac <bj||di> + d_ad <bj||ci> + d_bc <aj||di> - d_bd <aj||ci>
        nv = ev.size
        Iv, Io = np.eye(nv), np.eye(no)
        gvoov = g[v, o, v, o]  # <bj||di> as [b,j,d,i]
        K1 = ein("ij,abcd->abicdj", Io, g[v, v, v, v])
        K1 -= ein("ac,bjdi->abicdj", Iv, gvoov)
        K1 += ein("ad,bjci->abicdj", Iv, gvoov)
        K1 += ein("bc,ajdi->abicdj", Iv, gvoov)
        K1 -= ein("bd,ajci->abicdj", Iv, gvoov)
    return eps_so, M11, U, K1


def dense_matrix(eps_occ, eps_vir, B, level):
    """Spin-orbital ADC(level) matrix in the basis [1p a] + [2p1h (a<b, i)] ordered as
    a-major, then b, then i (the ordering of ``oracle.isr.ISR``)."""
    eps_so, M11, U, K1 = blocks(eps_occ, eps_vir, B, level)
    no = 2 * eps_occ.size
    nv = eps_so.size - no
    pairs = [(a, b) for a in range(nv) for b in range(nv) if a < b]
    cls2 = [(a, b, i) for (a, b) in pairs for i in range(no)]
    A = np.array([c[0] for c in cls2])
    Bb = np.array([c[1] for c in cls2])
    I = np.array([c[2] for c in cls2])
    n1, n2 = nv, len(cls2)
    M = np.zeros((n1 + n2, n1 + n2))
    M[:n1, :n1] = M11
    M[:n1, n1:] = U[:, A, Bb, I]
    M[n1:, :n1] = M[:n1, n1:].T
    ev, eo = eps_so[no:], eps_so[:no]
    M[n1:, n1:] = np.diag(ev[A] + ev[Bb] - eo[I])
    if K1 is not None:
        M[n1:, n1:] += K1[A[:, None], Bb[:, None], I[:, None], A[None, :], Bb[None, :], I[None, :]]
    return M


def doublet_embedding(nocc, nvir):
    """Columns: the closed-shell doublet (M_s = +1/2) basis in spin-orbital coordinates.

    Returns C with shape [n1_so + n2_so, nvir + nocc*nvir*nvir]: column a is the 1p
    state c+_{a alpha}; column (i, a, b) (z-coordinates, row-major i, a, b) is the
    2p1h state with D-coefficients x = z_S + z_A/sqrt(3) on c+_{a alpha} c+_{b beta}
    c_{i beta} Phi0 and y = x - x^T on the same-spin states c+_{a alpha} c+_{b alpha}
    c_{i alpha} Phi0 (a<b).  C^T C = 1."""
    no, nv = 2 * nocc, 2 * nvir
    pairs = [(a, b) for a in range(nv) for b in range(nv) if a < b]
    cls2 = {(a, b, i): k for k, (a, b, i) in enumerate([(a, b, i) for (a, b) in pairs for i in range(no)])}
    n1, n2 = nv, len(cls2)
    ncol = nvir + nocc * nvir * nvir
    C = np.zeros((n1 + n2, ncol))
    for a in range(nvir):
        C[2 * a, a] = 1.0
    s3 = np.sqrt(3.0)

    def put(col, A, Bv, I, val):
        # coefficient val on c+_A c+_Bv c_I Phi0 (spin-orbital virtual indices A,Bv)
        if A == Bv:
            return
        if A < Bv:
            C[n1 + cls2[(A, Bv, I)], col] += val
        else:
            C[n1 + cls2[(Bv, A, I)], col] -= val

    for i in range(nocc):
        for a in range(nvir):
            for b in range(nvir):
                col = nvir + (i * nvir + a) * nvir + b
                # unit z on (i,a,b): split into symmetric and antisymmetric parts
                zS = np.zeros((nvir, nvir))
                zA = np.zeros((nvir, nvir))
                e = np.zeros((nvir, nvir))
                e[a, b] = 1.0
                zS, zA = 0.5 * (e + e.T), 0.5 * (e - e.T)
                x = zS + zA / s3
                yy = x - x.T
                for c in range(nvir):
                    for d in range(nvir):
                        if x[c, d] != 0.0:
                            put(col, 2 * c, 2 * d + 1, 2 * i + 1, x[c, d])
                        if c < d and yy[c, d] != 0.0:
                            put(col, 2 * c, 2 * d, 2 * i, yy[c, d])
    return C
