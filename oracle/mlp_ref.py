"""FP64 NumPy reference of the learned Davidson preconditioner (forward, loss, gradients).

TEST INFRASTRUCTURE ONLY.

Per element e of a residual vector the network maps 6 features to one number u_e:
  x -> h1 = GELU(x W1 + b1) [256] -> h2 = GELU(h1 W2 + b2) [256] -> u = h2 W3 + b3,
GELU(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).  The preconditioned step is
t_e = a0_e (1 + u_e) with a0_e = r_e / (D_e - theta) the Jacobi (diagonal) step.
A training group g is a set of elements of one residual vector with the ideal
correction d_e (converged vector minus current Ritz vector, orthogonal to it);
its loss is the scale-free L_g = 1 - (a.d)^2 / ((a.a)(d.d)) with a_e = a0_e (1 + u_e),
and a batch loss is the mean over its groups.

Parameter layout (one flat array): W1[6][256], b1[256], W2[256][256], b2[256], W3[256], b3[1].
"""
import numpy as np

NF, H = 6, 256
SIZES = [("W1", (NF, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
C0 = np.sqrt(2.0 / np.pi)


def unpack(w):
    out, off = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(w[off:off + n], dtype=np.float64).reshape(shp)
        off += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C0 * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(C0 * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C0 * (1.0 + 3 * 0.044715 * z * z)


def forward(w, X):
    p = unpack(w)
    z1 = X @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    u = h2 @ p["W3"] + p["b3"][0]
    return u, (z1, h1, z2, h2)


def loss(w, X, a0, d, group):
    """Mean over groups (rows of an [ngroup, group] view) of 1 - cos^2(a, d)."""
    u, _ = forward(w, X)
    a = (a0 * (1.0 + u)).reshape(-1, group)
    dd = d.reshape(-1, group)
    pq = np.sum(a * dd, axis=1)
    q = np.sum(a * a, axis=1)
    n = np.sum(dd * dd, axis=1)
    return float(np.mean(1.0 - pq * pq / (q * n)))


def grad(w, X, a0, d, group):
    """Analytic gradient of ``loss`` with respect to the flat parameter vector."""
    p = unpack(w)
    u, (z1, h1, z2, h2) = forward(w, X)
    a = (a0 * (1.0 + u)).reshape(-1, group)
    dd = d.reshape(-1, group)
    G = a.shape[0]
    pq = np.sum(a * dd, axis=1, keepdims=True)
    q = np.sum(a * a, axis=1, keepdims=True)
    n = np.sum(dd * dd, axis=1, keepdims=True)
    dLda = -2.0 * pq / (q * n) * (dd - (pq / q) * a) / G
    du = dLda.reshape(-1) * a0
    g = {"W3": h2.T @ du, "b3": np.array([du.sum()])}
    dz2 = np.outer(du, p["W3"]) * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return np.concatenate([g[name].reshape(-1) for name, _ in SIZES])


def features(r, theta, D, eo, ev, nocc, nvir):
    """Per-element features of a residual vector r[v + o*v*v] for root theta (diagonal D).

    0: (D_e - theta) / (|theta| + 1)   1: r_e / rms(r)   2: 1 for 1p, 0 for 2p1h
    3: e_a   4: e_b (0 for 1p)   5: e_i (0 for 1p)."""
    v, o = nvir, nocc
    rms = np.sqrt(np.mean(r * r)) + 1e-300
    F = np.zeros((r.size, NF))
    F[:, 0] = (D - theta) / (abs(theta) + 1.0)
    F[:, 1] = r / rms
    F[:v, 2] = 1.0
    F[:v, 3] = ev
    idx = np.arange(o * v * v)
    i, a, b = idx // (v * v), (idx // v) % v, idx % v
    F[v:, 3] = ev[a]
    F[v:, 4] = ev[b]
    F[v:, 5] = eo[i]
    return F
