"""FP64 block Davidson for the lowest eigenpairs of a symmetric matrix given as sigma = M r.

TEST INFRASTRUCTURE ONLY.

Davidson's iterative diagonalisation with sigma vectors (Sec. "Algebraic
Diagrammatic Construction (ADC) Theory", last paragraph).  Plain textbook
version: orthonormal subspace V, Rayleigh-Ritz on V^T M V, residual
r = M x - theta x, diagonal (Jacobi) preconditioner (D - theta)^-1, two passes
of classical Gram-Schmidt, collapse onto the current Ritz vectors when the
subspace is full.

Readings where the paper is silent: guesses are unit vectors on the
nroots + 4 lowest diagonal entries (ties broken by index); a root is converged
when its residual 2-norm and its eigenvalue change since the previous
iteration are both <= conv.  When the subspace is full it restarts from the
lowest min(2*nroots + 2, max_space/2) Ritz vectors (thick restart).
"""
import numpy as np


def davidson(sigma, diag, nroots, conv=1e-6, max_iter=1000, max_space=None, guess=None, verbose=False):
    n = diag.size
    nguess = min(n, nroots + 4)
    if max_space is None:
        max_space = max(8 * nroots, 40)
    max_space = min(max_space, n)
    if guess is None:
        order = np.argsort(diag, kind="stable")[:nguess]
        V = np.zeros((nguess, n))
        V[np.arange(nguess), order] = 1.0
    else:
        V = np.linalg.qr(np.asarray(guess).T)[0].T
    S = sigma(V)
    theta_old = np.full(nroots, np.inf)
    it = 0
    while True:
        it += 1
        G = V @ S.T
        G = 0.5 * (G + G.T)
        wall, yall = np.linalg.eigh(G)
        w, y = wall[:nroots], yall[:, :nroots]
        X = y.T @ V
        R = y.T @ S - w[:, None] * X
        rn = np.linalg.norm(R, axis=1)
        done = (rn <= conv) & (np.abs(w - theta_old) <= conv)
        if verbose:
            print(it, w, rn)
        if done.all() or it >= max_iter:
            return w, X, rn, it, bool(done.all())
        theta_old = w
        new = []
        for k in np.where(~done)[0]:
            den = diag - w[k]
            den = np.where(np.abs(den) < 1e-8, np.copysign(1e-8, den), den)
            new.append(R[k] / den)
        new = np.array(new)
        # scale each correction to unit length first, so that the drop test below is relative
        new = new / np.maximum(np.linalg.norm(new, axis=1), 1e-300)[:, None]
        if V.shape[0] + new.shape[0] > max_space:
            nkeep = min(V.shape[0] - 1, max(nroots, min(2 * nroots + 2, max_space // 2)))
            yk = yall[:, :nkeep]
            V, S = yk.T @ V, yk.T @ S
        for _ in range(2):
            new = new - (new @ V.T) @ V
        keep = []
        for k in range(new.shape[0]):
            vk = new[k]
            for j in keep:
                vk = vk - (vk @ j) * j
            for j in keep:
                vk = vk - (vk @ j) * j
            nk = np.linalg.norm(vk)
            if nk > 1e-8:
                keep.append(vk / nk)
        if not keep:
            return w, X, rn, it, False
        keep = np.array(keep)
        V = np.vstack([V, keep])
        S = np.vstack([S, sigma(keep)])
