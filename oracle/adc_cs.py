"""Tier-2 oracle: closed-shell (spin-adapted) density-fitted EA-ADC(2)/ADC(3).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports this module.

Matrix-free sigma = M r on the doublet 1p + 2p1h space of a closed-shell
reference (Sec. "Algebraic Diagrammatic Construction (ADC) Theory", eqs 3-6;
Davidson sigma vectors as described there), with every two-electron integral
taken from the DF factor, (pq|rs) = sum_Q B^Q_pq B^Q_rs (eq 25).  Integrals with
at most two virtual indices are formed and kept; those with three or four
virtual indices are contracted through B on the fly (Sec. "Density Fitting (DF)
Approximation", last paragraph).

Coordinates.  r = (r1[a], z[i,a,b]).  z are orthonormal doublet coordinates of
the 2p1h space: with x = z_S + z_A/sqrt(3) the coefficients of the determinants
c+_{a alpha} c+_{b beta} c_{i beta} Phi0 and y = x - x^T those of
c+_{a alpha} c+_{b alpha} c_{i alpha} Phi0 (a<b), the state is a doublet and has
norm |r1|^2 + |z|^2.  A sigma vector is read off the alpha-beta determinants,
sigma_D, and returned as sigma_z = (sigma_D)_S + sqrt(3) (sigma_D)_A.

The closed forms are the spin-orbital ones of ``oracle.adc_so`` summed over spin
for a closed-shell reference; the result is pinned elementwise against
C^T M_so C (``oracle.adc_so.doublet_embedding``).

Notation (spatial orbitals): ovov[i,a,j,b] = (ia|jb), oovv[i,j,a,b] = (ij|ab),
oooo[i,j,k,l] = (ij|kl), ooov[i,j,k,a] = (ij|ka);
T[i,j,a,b] = (ia|jb) / (e_i + e_j - e_a - e_b) is the first-order amplitude
(alpha-beta block; the same-spin block is T - T^{ab-swapped}).
"""
import numpy as np

ein = lambda s, *a: np.einsum(s, *a, optimize=True)  # noqa: E731
SQ3 = np.sqrt(3.0)


def sym(x):
    """Symmetric part over the last two (virtual) axes."""
    return 0.5 * (x + np.swapaxes(x, -1, -2))


def asym(x):
    return 0.5 * (x - np.swapaxes(x, -1, -2))


def z_to_x(z):
    return sym(z) + asym(z) / SQ3


def d_to_z(s):
    return sym(s) + SQ3 * asym(s)


def ladder_rows(Bvv, amp, a_idx):
    """Selected rows of the ladder term: out[k, b] = sum_cd (ac|bd) amp[c, d] for a = a_idx[k], with
    (ac|bd) = sum_Q B^Q_ac B^Q_bd (eq 25) and amp [v, v] one 2p1h block.  For spot checks at sizes
    where whole rows of every vector are too dear: cost X v^2 per selected a."""
    out = np.empty((len(a_idx), Bvv.shape[1]))
    for k, a in enumerate(a_idx):
        W = Bvv[:, a, :] @ amp                      # [Q, d] = sum_c B^Q_ac amp_cd
        out[k] = np.einsum("Qd,Qbd->b", W, Bvv)     # sum_Q sum_d W[Q, d] B^Q_bd
    return out


class Problem:
    """Integrals and intermediates of one closed-shell instance."""

    def __init__(self, eps_occ, eps_vir, B):
        self.eo = np.asarray(eps_occ, float)
        self.ev = np.asarray(eps_vir, float)
        o, v = self.eo.size, self.ev.size
        self.o, self.v = o, v
        self.X = B.shape[0]
        self.Boo = np.ascontiguousarray(B[:, :o, :o])
        self.Bov = np.ascontiguousarray(B[:, :o, o:])
        self.Bvv = np.ascontiguousarray(B[:, o:, o:])
        # stored integrals: at most two virtual indices
        Lov = self.Bov.reshape(self.X, o * v)
        self.ovov = (Lov.T @ Lov).reshape(o, v, o, v)
        self.oovv = (self.Boo.reshape(self.X, o * o).T @ self.Bvv.reshape(self.X, v * v)).reshape(o, o, v, v)
        self.oooo = (self.Boo.reshape(self.X, o * o).T @ self.Boo.reshape(self.X, o * o)).reshape(o, o, o, o)
        self.ooov = (self.Boo.reshape(self.X, o * o).T @ Lov).reshape(o, o, o, v)
        self.D2 = (self.eo[:, None, None, None] + self.eo[None, :, None, None]
                   - self.ev[None, None, :, None] - self.ev[None, None, None, :])
        self.T = self.ovov.transpose(0, 2, 1, 3) / self.D2
        self._cache = {}

    # ------------------------------------------------------------------
    # on-the-fly integrals with three / four virtual indices
    # ------------------------------------------------------------------
    def vvvv_apply(self, amp):
        """sum_cd (ac|bd) amp[..., c, d] for amp[..., v, v] (the ladder).

        Small batches contract B directly, sum_Q B^Q amp B^Q; large batches form
        (ac|bd) for a block of a at a time and multiply."""
        v, X = self.v, self.X
        shp = amp.shape
        a2 = amp.reshape(-1, v, v)
        n = a2.shape[0]
        if X == 0:
            return np.zeros(shp)
        if 4 * X * n * v ** 3 <= 2 * X * v ** 4 + 2 * n * v ** 4:
            out = np.zeros_like(a2)
            for Q in range(X):
                BQ = self.Bvv[Q]
                out += BQ @ a2 @ BQ  # (B r B)_ab = sum_cd B_ac r_cd B_db, B symmetric
            return out.reshape(shp)
        out = np.empty((n, v, v))
        A = a2.reshape(n, v * v)
        Lvv = self.Bvv.reshape(X, v * v)
        ch = max(1, min(v, int(2.5e8 // (v ** 3))))
        for a0 in range(0, v, ch):
            a1 = min(v, a0 + ch)
            G = (self.Bvv[:, a0:a1, :].reshape(X, -1).T @ Lvv).reshape(a1 - a0, v, v, v)  # [a,c,b,d]
            G = G.transpose(0, 2, 1, 3).reshape((a1 - a0) * v, v * v)                       # [(a,b),(c,d)]
            out[:, a0:a1, :] = (A @ G.T).reshape(n, a1 - a0, v)
        return out.reshape(shp)

    # ------------------------------------------------------------------
    # ground-state quantities
    # ------------------------------------------------------------------
    def mp2_energy(self):
        """E_MP2 = sum T^{ab}_ij [2 (ia|jb) - (ib|ja)]."""
        g = self.ovov.transpose(0, 2, 1, 3)
        return float(np.sum(self.T * (2.0 * g - g.transpose(0, 1, 3, 2))))

    def second_order(self):
        """Second-order doubles residual Y (alpha-beta), amplitudes U2 = Y/D and singles u1."""
        if "so" in self._cache:
            return self._cache["so"]
        T, ovov, oovv, oooo = self.T, self.ovov, self.oovv, self.oooo
        Tt = T.transpose(0, 1, 3, 2)  # T^{ba}_{ij}
        L = self.vvvv_apply(T)                                   # sum_cd (ac|bd) T^cd_ij
        H = ein("klab,kilj->ijab", T, oooo)                      # sum_kl T^ab_kl (ki|lj)
        R1 = ein("ikac,jbkc->ijab", 2.0 * T - Tt, ovov) - ein("ikac,kjbc->ijab", T, oovv)
        R2 = -ein("kjac,kibc->ijab", T, oovv)
        R3 = -ein("ikcb,kjac->ijab", T, oovv)
        R4 = ein("jkbc,iakc->ijab", 2.0 * T - Tt, ovov) - ein("jkbc,kiac->ijab", T, oovv)
        Y = L + H + R1 + R2 + R3 + R4
        U2 = Y / self.D2
        # singles: sum_kcd (2T^cd_ik - T^dc_ik)(ac|kd) - sum_klc (2T^ac_kl - T^ca_kl)(ki|lc)
        Tt_ = 2.0 * T - Tt
        W = ein("Qkd,ikcd->Qic", self.Bov, Tt_)                 # sum_kd (Q|kd) Ttilde^cd_ik
        y1 = ein("Qac,Qic->ia", self.Bvv, W)
        y1 -= ein("klac,kilc->ia", Tt_, self.ooov.transpose(0, 1, 2, 3))
        u1 = y1 / (self.eo[:, None] - self.ev[None, :])
        self._cache["so"] = (L, Y, U2, u1)
        return self._cache["so"]

    def mp2_density_vv(self):
        """Per-spin MP2 virtual-virtual density D_ed = sum_klc (2T^ce_kl - T^ec_kl) T^cd_kl."""
        T = self.T
        return ein("klce,klcd->ed", 2.0 * T - T.transpose(0, 1, 3, 2), T)

    def mp2_density_oo(self):
        """Per-spin MP2 occupied-occupied density D_ml = -sum_kcd (2T^cd_mk - T^dc_mk) T^cd_lk."""
        T = self.T
        return -ein("mkcd,lkcd->ml", 2.0 * T - T.transpose(0, 1, 3, 2), T)

    # ------------------------------------------------------------------
    # secular-matrix pieces
    # ------------------------------------------------------------------
    def _pm2(self, A):
        """P_ab = sum_ckl (2A^ac_kl - A^ca_kl)(kb|lc); returns -(P + P^T)/2."""
        P = ein("klac,kblc->ab", 2.0 * A - A.transpose(0, 1, 3, 2), self.ovov)
        return -0.5 * (P + P.T)

    def fock_like(self, rho_oo, rho_vv, rho_ov):
        """sum_pq <ap||bq> rho_pq for a spin-diagonal density (static self-energy)."""
        Boo, Bov, Bvv = self.Boo, self.Bov, self.Bvv
        J = ein("Qml,ml->Q", Boo, rho_oo) + ein("Qed,ed->Q", Bvv, rho_vv) + 2.0 * ein("Qkc,kc->Q", Bov, rho_ov)
        out = 2.0 * ein("Qab,Q->ab", Bvv, J)
        # exchange: (al|mb) rho_ml, (ad|eb) rho_ed, (ak|bc)+(ac|bk) rho_kc
        out -= ein("Qma,ml,Qlb->ab", Bov, rho_oo, Bov)
        out -= ein("Qad,ed,Qeb->ab", Bvv, rho_vv, Bvv)
        Z = ein("Qbc,kc->Qkb", Bvv, rho_ov)
        out -= ein("Qka,Qkb->ab", Bov, Z)
        out -= ein("Qkb,Qka->ab", Bov, Z)
        return out

    def m11(self, level):
        """1p-1p block M11 [v, v] (ADC(2): through 2nd order; ADC(3): through 3rd)."""
        key = ("m11", level)
        if key in self._cache:
            return self._cache[key]
        T = self.T
        M = np.diag(self.ev) + self._pm2(T)
        if level >= 3:
            L, Y, U2, u1 = self.second_order()
            # static self-energy with the second-order density (oo, vv and ov blocks)
            M += self.fock_like(self.mp2_density_oo(), self.mp2_density_vv(), u1)
            # second-order form with second-order amplitudes
            M += self._pm2(U2)
            # ladder part of the remaining first-order amplitude products
            Lt = 2.0 * L - L.transpose(0, 1, 3, 2)
            Q = ein("klae,klbe->ab", T, Lt)
            M -= 0.5 * (Q + Q.T)
            # ring part
            Tt = T.transpose(0, 1, 3, 2)
            dbml = self.oovv.transpose(2, 3, 0, 1)               # (db|ml) as [d,b,m,l]
            dlmb = self.ovov.transpose(1, 0, 2, 3)               # (dl|mb) as [d,l,m,b]
            g1 = ein("dbml->dlbm", dbml) - ein("dlmb->dlbm", dlmb)  # (db|ml) - (dl|mb)
            g2 = ein("dlmb->dlbm", dlmb)                             # (dl|mb)
            RA = ein("klcd,dlbm->ckbm", T - Tt, g1) - ein("klcd,dlbm->ckbm", T, g2)
            RB = ein("klcd,dlbm->ckbm", T, g1) - ein("klcd,dlbm->ckbm", T - Tt, g2)
            RC = -ein("kldc,dlbm->ckbm", T, ein("dbml->dlbm", dbml))
            Rg = (ein("kmac,ckbm->ab", T - Tt, RA) - ein("mkac,ckbm->ab", T, RB)
                  + ein("kmac,ckbm->ab", T, RC))
            M -= 0.5 * (Rg + Rg.T)
        self._cache[key] = M
        return M

    def coupling_D(self, level):
        """U_D[a,b,c,i]: coupling of 1p a (alpha) to c+_{b alpha} c+_{c beta} c_{i beta} Phi0."""
        key = ("uD", level)
        if key in self._cache:
            return self._cache[key]
        U = ein("Qab,Qic->abci", self.Bvv, self.Bov)              # (ab|ic)
        if level >= 3:
            T = self.T
            Tt = T.transpose(0, 1, 3, 2)
            o, v = self.o, self.v
            # sum_kl T^bc_kl (ak|il), with (ak|il) = ooov[i,l,k,a]
            U += ein("klbc,ilka->abci", T, self.ooov)
            # (ka|cd) for all k, a, c, d, formed once
            ovvv = (self.Bov.reshape(self.X, o * v).T @ self.Bvv.reshape(self.X, v * v)).reshape(o, v, v, v)
            # -sum_kd T^bd_ki (ak|cd):  [(i,b),(k,d)] x [(k,d),(a,c)]
            A = T.transpose(1, 2, 0, 3).reshape(o * v, o * v)
            G = ovvv.transpose(0, 3, 1, 2).reshape(o * v, v * v)
            U -= (A @ G).reshape(o, v, v, v).transpose(2, 1, 3, 0)
            # +sum_kd (2T^cd_ik - T^dc_ik)(ab|kd):  [(i,c),(k,d)] x [(k,d),(a,b)]
            A = (2.0 * T - Tt).transpose(0, 2, 1, 3).reshape(o * v, o * v)
            G = ovvv.reshape(o * v, v * v)
            U += (A @ G).reshape(o, v, v, v).transpose(2, 3, 1, 0)
            # -sum_kd T^cd_ik (ak|bd):  [(i,c),(k,d)] x [(k,d),(a,b)]
            A = T.transpose(0, 2, 1, 3).reshape(o * v, o * v)
            G = ovvv.transpose(0, 3, 1, 2).reshape(o * v, v * v)
            U -= (A @ G).reshape(o, v, v, v).transpose(2, 3, 1, 0)
            del ovvv, G, A
        self._cache[key] = U
        return U

    def coupling_z(self, level):
        """U_z[a,i,b,c] = [(U_D)_S + sqrt(3) (U_D)_A] over (b,c): the 1p-2p1h block in z."""
        key = ("uz", level)
        if key not in self._cache:
            self._cache[key] = d_to_z(self.coupling_D(level).transpose(0, 3, 1, 2))
        return self._cache[key]

    def k0(self):
        return (self.ev[None, :, None] + self.ev[None, None, :] - self.eo[:, None, None])

    def k1_D(self, x):
        """First-order 2p1h-2p1h term on the alpha-beta determinants, x[..., i,a,b] -> sigma_D.

        sum_cd (ac|bd) x_cdi - sum_dj (bd|ij) x_adj - sum_dj (ad|ij) x_dbj
        + sum_dj (bi|jd) (2 x_adj - x_daj)."""
        s = self.vvvv_apply(x)
        s -= ein("ijbd,...jad->...iab", self.oovv, x)
        s -= ein("ijad,...jdb->...iab", self.oovv, x)
        s += ein("ibjd,...jad->...iab", self.ovov, 2.0 * x - np.swapaxes(x, -1, -2))
        return s

    # ------------------------------------------------------------------
    # sigma, diagonal, dense matrix
    # ------------------------------------------------------------------
    def dim(self):
        return self.v + self.o * self.v * self.v

    def split(self, r):
        r = np.asarray(r)
        return r[..., :self.v], r[..., self.v:].reshape(r.shape[:-1] + (self.o, self.v, self.v))

    def sigma(self, r, level):
        """sigma = M r for r[..., v + o*v*v] (one vector or a stack)."""
        r1, z = self.split(r)
        M11, Uz = self.m11(level), self.coupling_z(level)
        s1 = r1 @ M11.T + ein("aibc,...ibc->...a", Uz, z)
        s2 = ein("aibc,...a->...ibc", Uz, r1) + self.k0() * z
        if level >= 3:
            s2 = s2 + d_to_z(self.k1_D(z_to_x(z)))
        return np.concatenate([s1, s2.reshape(s2.shape[:-3] + (-1,))], axis=-1)

    def diagonal(self, level):
        """Diagonal of M in the (r1, z) coordinates."""
        d1 = np.diag(self.m11(level))
        d2 = self.k0().copy()
        if level >= 3:
            o, v = self.o, self.v
            aabb = ein("Qaa,Qbb->ab", self.Bvv, self.Bvv)           # (aa|bb)
            abab = ein("Qab,Qab->ab", self.Bvv, self.Bvv)           # (ab|ab)
            aaii = ein("iiaa->ia", self.oovv)                        # (aa|ii)
            aiia = ein("iaia->ia", self.ovov)                        # (ai|ia)
            Kabab = aabb[None] - aaii[:, None, :] - aaii[:, :, None] + 2.0 * aiia[:, None, :]
            Kbaba = aabb[None] - aaii[:, :, None] - aaii[:, None, :] + 2.0 * aiia[:, :, None]
            Kabba = abab[None] - aiia[:, None, :]                    # (ab|ab) - (bi|ib)
            Kbaab = abab[None] - aiia[:, :, None]                    # (ab|ab) - (ai|ia)
            al, be = 0.5 + SQ3 / 2, 0.5 - SQ3 / 2
            ga, de = 0.5 + 0.5 / SQ3, 0.5 - 0.5 / SQ3
            dK = al * ga * Kabab + al * de * Kabba + be * ga * Kbaab + be * de * Kbaba
            idx = np.arange(v)
            dK[:, idx, idx] = (ein("Qaa,Qaa->a", self.Bvv, self.Bvv)[None, :]
                               - 2.0 * aaii + aiia)
            d2 = d2 + dK
        return np.concatenate([d1, d2.reshape(-1)])

    def dense(self, level):
        n = self.dim()
        return self.sigma(np.eye(n), level)

    # ------------------------------------------------------------------
    # spectral amplitudes (eqs 7-8): x = Y^T f, f_Ap = <Psi~_A| c+_p |Psi0>, p an alpha spin-orbital
    # (the doublet states here have M_s = +1/2).  f is kept through second order in the 1p block and
    # first order in the 2p1h block (the orders of ADC(2)'s transition amplitudes); its closed forms
    # were read off the intermediate states of tier 0 order by order:
    #   f[a, b] = delta_ab - D^MP2_ab / 2           (b virtual; D per spin)
    #   f[a, j] = -u1[j, a]                          (j occupied; u1 the second-order singles)
    #   f[(i,a,b), j] = -(S + sqrt3 A)(T[j,i])_ab    (z coordinates; no first-order part for virtual p)
    # ------------------------------------------------------------------
    def transition_amplitudes(self):
        """f[N, o + v]: rows in (r1, z) coordinates, columns the spatial orbitals (occupied first)."""
        o, v = self.o, self.v
        f = np.zeros((self.dim(), o + v))
        f[:v, o:] = np.eye(v) - 0.5 * self.mp2_density_vv()
        f[:v, :o] = -self.second_order()[3].T
        for j in range(o):
            f[v:, j] = -d_to_z(self.T[j]).reshape(-1)   # T[j][i, a, b] = T^ab_ji
        return f

    def spectral_amplitudes(self, vecs):
        """x[k, p] = sum_A Y[k, A] f[A, p] for eigenvectors vecs[k] (eq 7)."""
        return np.asarray(vecs) @ self.transition_amplitudes()

    # ------------------------------------------------------------------
    # scaled-matrix ADC (Sec. "ADC Theory", the equation after eq 5): the paper states that x = 0
    # gives ADC(2) and x = 1 ADC(3); its formula M0 + M1 + M2 + x M3 taken literally would keep the
    # second-order coupling and the first-order 2p1h terms at x = 0, so the reading is
    # M_sm = M_ADC(2) + x (M_ADC(3) - M_ADC(2)), which meets both statements.
    # ------------------------------------------------------------------
    def sigma_sm(self, r, x):
        s2 = self.sigma(r, 2)
        return s2 + x * (self.sigma(r, 3) - s2)

    def diagonal_sm(self, x):
        d2 = self.diagonal(2)
        return d2 + x * (self.diagonal(3) - d2)

    def dense_sm(self, x):
        return self.sigma_sm(np.eye(self.dim()), x)
