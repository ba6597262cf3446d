"""Tier-0 oracle: the EA-ADC secular matrix built numerically from its definition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module.

What is computed (Sec. "Algebraic Diagrammatic Construction (ADC) Theory",
eqs 1-6 and eq 5):

* A closed-shell N-electron problem in spin-orbitals with canonical Hartree-Fock
  orbital energies eps (Fock = diag(eps)) and two-electron integrals from the DF
  factor, (pq|rs) = sum_Q B^Q_pq B^Q_rs (eq 25).  The one-electron operator h is
  chosen so that the Fock matrix of the doubly occupied reference is diag(eps).
* The Moller-Plesset partition H(lam) = H0 + lam*W, H0 = sum_p eps_p n_p.
* The ground state Psi0(lam) and E0(lam) from Rayleigh-Schroedinger perturbation
  theory, carried as truncated power series in lam (intermediate normalisation;
  the intermediate states below do not depend on the norm of Psi0).
* The intermediate states exactly as the ISR construction describes them:
  class 1 precursors c+_a Psi0; class 2 precursors c+_a c+_b c_i Psi0 (a<b),
  first Gram-Schmidt orthogonalised against the class-1 states, then each class
  symmetrically (Loewdin) orthonormalised, S^-1/2 taken as a power series.
* M(lam) = <Psi~_A | H - E0 | Psi~_B> (eq 3) as a power series.  ADC(n) keeps
  M11 through order n, M12 through order n-1 and M22 through order n-2 for n=2
  and order 1 for n=3 (eq 5 truncated; the usual order relations of the
  1p/2p1h blocks).

Everything is exact power-series arithmetic in float64: no finite differences.
Sizes: a handful of occupied and virtual orbitals (the determinant spaces are
held densely).

Basis conventions used by every spin-orbital routine in this package:
  spin-orbital index P = 2*p + s (p spatial, s = 0 alpha, 1 beta);
  occupied spin-orbitals 0..2o-1, virtual 2o..2n-1;
  1p state  |a>    = c+_a |Phi0>;
  2p1h state |abi> = c+_a c+_b c_i |Phi0> with a < b (operators act right to left).
"""
import itertools
import numpy as np
import scipy.sparse as sp

ORDER = 3  # highest power of lambda carried


# ----------------------------------------------------------------------------
# integrals in spin-orbital form
# ----------------------------------------------------------------------------
def spatial_eri(B):
    """(pq|rs) = sum_Q B^Q_pq B^Q_rs (eq 25), dense [n,n,n,n]."""
    return np.einsum("Qpq,Qrs->pqrs", B, B)


def spin_orbital_tensors(eps_occ, eps_vir, B):
    """Return (eps_so[2n], asym[2n,2n,2n,2n]) with asym[p,q,r,s] = <pq||rs>."""
    eps = np.concatenate([eps_occ, eps_vir])
    n = eps.size
    g = spatial_eri(B)
    eps_so = np.repeat(eps, 2)
    spin = np.tile([0, 1], n)
    sp_ = np.repeat(np.arange(n), 2)
    # <pq|rs> = (pr|qs) delta(s_p,s_r) delta(s_q,s_s)
    phys = g[np.ix_(sp_, sp_, sp_, sp_)].transpose(0, 2, 1, 3)
    same_pr = spin[:, None] == spin[None, :]
    phys = phys * same_pr[:, None, :, None] * same_pr[None, :, None, :]
    asym = phys - phys.transpose(0, 1, 3, 2)
    return eps_so, asym


# ----------------------------------------------------------------------------
# determinant spaces
# ----------------------------------------------------------------------------
class FockSpace:
    """All determinants with ``nelec`` electrons in ``norb`` spin-orbitals."""

    def __init__(self, norb, nelec):
        self.norb, self.nelec = norb, nelec
        dets = []
        for occ in itertools.combinations(range(norb), nelec):
            d = 0
            for p in occ:
                d |= 1 << p
            dets.append(d)
        self.dets = np.array(dets, dtype=np.int64)
        self.index = {int(d): k for k, d in enumerate(dets)}
        self.dim = len(dets)


def _popcount_below(d, p):
    return bin(d & ((1 << p) - 1)).count("1")


class Ladder:
    """c_p : space(n) -> space(n-1) and c+_p : space(n) -> space(n+1) as index maps."""

    def __init__(self, spaces):
        self.spaces = spaces  # dict nelec -> FockSpace
        self._ann, self._cre = {}, {}

    def ann(self, p, n):
        key = (p, n)
        if key not in self._ann:
            src, dst, sgn = [], [], []
            S, D = self.spaces[n], self.spaces[n - 1]
            for k, d in enumerate(S.dets):
                d = int(d)
                if d >> p & 1:
                    src.append(k)
                    dst.append(D.index[d ^ (1 << p)])
                    sgn.append(-1.0 if _popcount_below(d, p) % 2 else 1.0)
            self._ann[key] = (np.array(src, int), np.array(dst, int), np.array(sgn))
        return self._ann[key]

    def cre(self, p, n):
        key = (p, n)
        if key not in self._cre:
            src, dst, sgn = [], [], []
            S, D = self.spaces[n], self.spaces[n + 1]
            for k, d in enumerate(S.dets):
                d = int(d)
                if not (d >> p & 1):
                    src.append(k)
                    dst.append(D.index[d | (1 << p)])
                    sgn.append(-1.0 if _popcount_below(d, p) % 2 else 1.0)
            self._cre[key] = (np.array(src, int), np.array(dst, int), np.array(sgn))
        return self._cre[key]

    def apply(self, kind, p, n, vec):
        """Apply c_p ('a') or c+_p ('c') to vec[..., dim(n)]."""
        src, dst, sgn = (self.ann if kind == "a" else self.cre)(p, n)
        n_out = n - 1 if kind == "a" else n + 1
        out = np.zeros(vec.shape[:-1] + (self.spaces[n_out].dim,))
        out[..., dst] = vec[..., src] * sgn
        return out

    def one_body(self, p, q, n):
        """Sparse matrix of c+_p c_q on space(n)."""
        s1, d1, g1 = self.ann(q, n)
        dim = self.spaces[n].dim
        A = sp.csr_matrix((g1, (d1, s1)), shape=(self.spaces[n - 1].dim, dim))
        s2, d2, g2 = self.cre(p, n - 1)
        C = sp.csr_matrix((g2, (d2, s2)), shape=(dim, self.spaces[n - 1].dim))
        return C @ A


def hamiltonian(eps_occ, eps_vir, B, ladder, n):
    """(H0 diagonal, W dense) on space(n).

    H = sum_pq k_pq E_pq + 1/2 sum_Q (L^Q)^2, L^Q = sum_pq B^Q_pq E_pq (spin-summed
    E_pq), which is the usual two-body operator written with the DF factor.  The
    one-electron part is h = diag(eps) - sum_i [2(pq|ii) - (pi|iq)] so that the
    reference Fock matrix is diag(eps)."""
    nocc = eps_occ.size
    eps = np.concatenate([eps_occ, eps_vir])
    norb = eps.size
    g = spatial_eri(B)
    occ = np.arange(nocc)
    h = np.diag(eps) - (2.0 * np.einsum("pqii->pq", g[:, :, occ][:, :, :, occ])
                        - np.einsum("piiq->pq", g[:, occ][:, :, occ]))
    k = h - 0.5 * np.einsum("pqqs->ps", g)
    S = ladder.spaces[n]
    E = {}
    for p in range(norb):
        for q in range(norb):
            E[p, q] = ladder.one_body(2 * p, 2 * q, n) + ladder.one_body(2 * p + 1, 2 * q + 1, n)
    H = sp.csr_matrix((S.dim, S.dim))
    for p in range(norb):
        for q in range(norb):
            if k[p, q] != 0.0:
                H = H + k[p, q] * E[p, q]
    for Q in range(B.shape[0]):
        L = sp.csr_matrix((S.dim, S.dim))
        for p in range(norb):
            for q in range(norb):
                if B[Q, p, q] != 0.0:
                    L = L + B[Q, p, q] * E[p, q]
        H = H + 0.5 * (L @ L)
    H = H.toarray()
    eps_so = np.repeat(eps, 2)
    h0 = np.array([sum(eps_so[p] for p in range(2 * norb) if int(d) >> p & 1) for d in S.dets])
    W = H - np.diag(h0)
    return h0, W


# ----------------------------------------------------------------------------
# power series helpers (axis 0 = order)
# ----------------------------------------------------------------------------
def s_mul(a, b, op):
    """Truncated product of two series; op(x, y) is the per-order product."""
    K = ORDER
    out = None
    for n in range(K + 1):
        acc = None
        for k in range(n + 1):
            t = op(a[k], b[n - k])
            acc = t if acc is None else acc + t
        out = acc[None] if out is None else np.concatenate([out, acc[None]])
    return out


def s_inv_sqrt(S):
    """(I + X)^(-1/2) for a matrix series with S[0] = I."""
    K = ORDER
    X = S.copy()
    X[0] = 0.0
    eye = np.zeros_like(S)
    eye[0] = np.eye(S.shape[1])
    out = eye.copy()
    term = eye.copy()
    coef = 1.0
    for k in range(1, K + 1):
        term = s_mul(term, X, lambda x, y: x @ y)
        coef *= (-0.5 - (k - 1)) / k
        out = out + coef * term
    return out


# ----------------------------------------------------------------------------
# the ISR secular matrix
# ----------------------------------------------------------------------------
class ISR:
    """Numerical intermediate-state representation of EA-ADC for a tiny problem."""

    def __init__(self, eps_occ, eps_vir, B):
        self.o, self.v = eps_occ.size, eps_vir.size
        norb = 2 * (self.o + self.v)
        N = 2 * self.o
        self.N = N
        spaces = {m: FockSpace(norb, m) for m in (N - 1, N, N + 1)}
        self.lad = Ladder(spaces)
        self.h0N, self.WN = hamiltonian(eps_occ, eps_vir, B, self.lad, N)
        self.h0P, self.WP = hamiltonian(eps_occ, eps_vir, B, self.lad, N + 1)
        self.occ = list(range(N))
        self.vir = list(range(N, norb))
        self.pairs = [(a, b) for a in self.vir for b in self.vir if a < b]
        self.class2 = [(a, b, i) for (a, b) in self.pairs for i in self.occ]
        self._ground_state()
        self._build()

    # Rayleigh-Schroedinger series for Psi0 and E0
    def _ground_state(self):
        S = self.lad.spaces[self.N]
        ref = S.index[(1 << self.N) - 1]
        e00 = self.h0N[ref]
        denom = e00 - self.h0N
        denom[ref] = np.inf
        psi = np.zeros((ORDER + 1, S.dim))
        psi[0, ref] = 1.0
        E = np.zeros(ORDER + 1)
        E[0] = e00
        for n in range(1, ORDER + 1):
            E[n] = (self.WN @ psi[n - 1])[ref]
            rhs = self.WN @ psi[n - 1]
            for k in range(1, n + 1):
                rhs = rhs - E[k] * psi[n - k]
            psi[n] = rhs / denom
        self.psi0, self.E0 = psi, E

    def _apply_string(self, ops, vec, n):
        """ops applied right to left, e.g. [('c',a),('c',b),('a',i)] = c+_a c+_b c_i."""
        for kind, p in reversed(ops):
            vec = self.lad.apply(kind, p, n, vec)
            n = n - 1 if kind == "a" else n + 1
        return vec

    def _hmE(self, vec):
        """(H(lam) - E0(lam)) applied to a series of (N+1)-electron vectors vec[k, m, dim]."""
        out = np.zeros_like(vec)
        e00 = self.E0[0]
        for n in range(ORDER + 1):
            acc = (self.h0P - e00) * vec[n]
            if n >= 1:
                acc = acc + vec[n - 1] @ self.WP.T
            for k in range(1, n + 1):
                acc = acc - self.E0[k] * vec[n - k]
            out[n] = acc
        return out

    def _build(self):
        N = self.N
        dot = lambda x, y: x @ y.T  # noqa: E731  rows are states
        # class 1
        P1 = np.stack([self._apply_string([("c", a)], self.psi0, N) for a in self.vir], axis=1)
        S1 = s_mul(P1, P1, dot)
        T1 = s_inv_sqrt(S1)
        Y1 = s_mul(T1.transpose(0, 2, 1), P1, lambda x, y: x @ y)
        # class 2 precursors, Gram-Schmidt against class 1
        P2 = np.stack([self._apply_string([("c", a), ("c", b), ("a", i)], self.psi0, N)
                       for (a, b, i) in self.class2], axis=1)
        ov = s_mul(Y1, P2, dot)  # [n1, n2] = <Y1|P2>
        P2 = P2 - s_mul(ov.transpose(0, 2, 1), Y1, lambda x, y: x @ y)
        S2 = s_mul(P2, P2, dot)
        T2 = s_inv_sqrt(S2)
        Y2 = s_mul(T2.transpose(0, 2, 1), P2, lambda x, y: x @ y)
        Y = np.concatenate([Y1, Y2], axis=1)
        HY = self._hmE(Y)
        self.M = s_mul(Y, HY, dot)  # M[k] = order-k coefficient
        self.n1 = len(self.vir)
        self.Y = Y

    def adc_matrix(self, level, lam=1.0, orders=None):
        """Strict ADC(level) matrix (level 2 or 3) at coupling lam.

        orders overrides the (M11, M12, M22) truncation orders."""
        if orders is None:
            orders = {2: (2, 1, 0), 3: (3, 2, 1)}[level]
        n1 = self.n1
        out = np.zeros(self.M.shape[1:])
        blocks = [(slice(0, n1), slice(0, n1), orders[0]),
                  (slice(0, n1), slice(n1, None), orders[1]),
                  (slice(n1, None), slice(0, n1), orders[1]),
                  (slice(n1, None), slice(n1, None), orders[2])]
        for r, c, kmax in blocks:
            for k in range(kmax + 1):
                out[r, c] += lam ** k * self.M[k][r, c]
        return out

    # brute force references
    def fci_ea(self, lam=1.0, nstates=None):
        """Exact EA-type excitation energies E_k(N+1) - E_0(N) of H0 + lam*W."""
        HN = np.diag(self.h0N) + lam * self.WN
        HP = np.diag(self.h0P) + lam * self.WP
        e0 = np.linalg.eigvalsh(HN)[0]
        eP = np.linalg.eigvalsh(HP)
        return eP - e0
