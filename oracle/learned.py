"""FP64 oracle of the learned block preconditioner for PCG on the reduced pose
system S dtheta = -b (test infrastructure: only the tests, the smoke check and
the benchmark's CPU baseline use this module).

The paper solves the reduced system by inverting H once (IC, Sec. 3.5) or by
factorizing it every iteration (FC, Sec. 1); it has no iterative solver and no
learned component, so this part is project-defined. Definitions:

* Block whitening. S has 6x6 blocks S_ij (one block row per frame). With the
  Cholesky factor S_ii = C_i C_i^T, the whitened system is
  S^ = D S D^T, D = blockdiag(C_i^{-1}); its diagonal blocks are I and its
  off-diagonal blocks S^_ij = C_i^{-1} S_ij C_j^{-T}. The coupling of block i
  is G_i = sum_{j != i} S^_ij S^_ij^T (so that (S^ S^)_ii = I + G_i).
* Features of block i (22 values): the upper triangle (row-major) of
  G_i / (1 + tr G_i) and log(1 + tr G_i).
* Network: x -> relu(W1 x + b1) -> relu(W2 h1 + b2) -> y = W3 h2 + b3,
  with 22 -> 256 -> 256 -> 21 units.
* Output: y (21 values) is the lower triangle (row-major) of a 6x6 factor L
  with L_kk = exp(y_kk); the whitened block preconditioner is P^ = L L^T and
  the block of M^{-1} is P_i = C_i^{-T} P^_i C_i^{-1}. A zero output gives
  P^ = I, i.e. block Jacobi (P_i = S_ii^{-1}).
* Training loss of block i: l_i = tr(P^ A P^) - 2 tr(P^) + 6, A = I + G_i,
  which is E ||P^ (S^ z)_i - z_i||^2 for z ~ N(0, I) (the block row of the
  Frobenius distance ||P S^ - I|| of sparse approximate inverses); it is
  minimized by P^ = A^{-1}. The batch loss is the mean over blocks.
* PCG: the textbook preconditioned conjugate gradient iteration with
  M^{-1} = blockdiag(P_i), started from x = 0, stopped when
  ||b - S x|| <= tol ||b||.
"""
import numpy as np

N_IN, N_HID, N_OUT = 22, 256, 21
TRI = [(r, c) for r in range(6) for c in range(r + 1)]          # lower triangle, row-major
UPPER = [(r, c) for r in range(6) for c in range(r, 6)]         # upper triangle, row-major
PARAM_SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
                ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def block_whitening(S):
    """C (nb, 6, 6) Cholesky factors of the diagonal blocks, Ci = C^{-1}, and the
    couplings G (nb, 6, 6) of the whitened system."""
    n = S.shape[0]
    nb = n // 6
    C = np.stack([np.linalg.cholesky(S[6 * i:6 * i + 6, 6 * i:6 * i + 6]) for i in range(nb)])
    Ci = np.stack([np.linalg.inv(c) for c in C])
    G = np.zeros((nb, 6, 6))
    for i in range(nb):
        for j in range(nb):
            if j != i:
                Sh = Ci[i] @ S[6 * i:6 * i + 6, 6 * j:6 * j + 6] @ Ci[j].T
                G[i] += Sh @ Sh.T
    return C, Ci, G


def features(G):
    """(nb, 22) network inputs of the blocks."""
    tr = np.trace(G, axis1=1, axis2=2)
    up = np.stack([G[:, r, c] for r, c in UPPER], axis=1)
    return np.concatenate([up / (1.0 + tr)[:, None], np.log1p(tr)[:, None]], axis=1)


def init_params(seed):
    """He-scaled hidden layers; the output layer starts at zero (block Jacobi)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0.0, np.sqrt(2.0 / N_IN), (N_HID, N_IN)), "b1": np.zeros(N_HID),
         "W2": rng.normal(0.0, np.sqrt(2.0 / N_HID), (N_HID, N_HID)), "b2": np.zeros(N_HID),
         "W3": np.zeros((N_OUT, N_HID)), "b3": np.zeros(N_OUT)}
    return p


def pack(p):
    return np.concatenate([p[k].reshape(-1) for k, _ in PARAM_SHAPES])


def unpack(v):
    p, o = {}, 0
    for k, s in PARAM_SHAPES:
        m = int(np.prod(s))
        p[k] = np.asarray(v[o:o + m], float).reshape(s)
        o += m
    return p


def mlp_forward(p, X):
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    Y = h2 @ p["W3"].T + p["b3"]
    return Y, (X, z1, h1, z2, h2)


def mlp_backward(p, cache, dY):
    X, z1, h1, z2, h2 = cache
    g = {"W3": dY.T @ h2, "b3": dY.sum(0)}
    d2 = (dY @ p["W3"]) * (z2 > 0)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"], g["b1"] = d1.T @ X, d1.sum(0)
    return g


def factor_from_output(Y):
    """(nb, 6, 6) lower factors L from network outputs (exp on the diagonal)."""
    L = np.zeros((Y.shape[0], 6, 6))
    for k, (r, c) in enumerate(TRI):
        L[:, r, c] = np.exp(Y[:, k]) if r == c else Y[:, k]
    return L


def block_loss(Y, G):
    """Per-block losses l_i and dl_i / dY (nb, 21)."""
    L = factor_from_output(Y)
    P = L @ np.swapaxes(L, 1, 2)
    A = np.eye(6)[None] + G
    PA = P @ A
    loss = np.einsum("bij,bji->b", PA, P) - 2.0 * np.trace(P, axis1=1, axis2=2) + 6.0
    dP = 2.0 * PA - 2.0 * np.eye(6)[None]          # d l / d P for P used as a general matrix
    dL = (dP + np.swapaxes(dP, 1, 2)) @ L            # P = L L^T
    dY = np.zeros_like(Y)
    for k, (r, c) in enumerate(TRI):
        dY[:, k] = dL[:, r, c] * (L[:, r, c] if r == c else 1.0)
    return loss, dY


def loss_and_grads(p, X, G):
    """Mean block loss over the batch and its gradient with respect to the parameters."""
    Y, cache = mlp_forward(p, X)
    loss, dY = block_loss(Y, G)
    nb = X.shape[0]
    g = mlp_backward(p, cache, dY / nb)
    return float(loss.mean()), g


def learned_blocks(p, S):
    """Blocks P_i of the learned M^{-1} for the system S."""
    C, Ci, G = block_whitening(S)
    Y, _ = mlp_forward(p, features(G))
    L = factor_from_output(Y)
    Ph = L @ np.swapaxes(L, 1, 2)
    return np.swapaxes(Ci, 1, 2) @ Ph @ Ci


def optimal_blocks(S):
    """Blocks P_i of M^{-1} at the minimizer of the training loss itself:
    P^_i = (I + G_i)^{-1}, so P_i = C_i^{-T} (I + G_i)^{-1} C_i^{-1} (the
    lowest block loss any network output can reach)."""
    C, Ci, G = block_whitening(S)
    Ph = np.linalg.inv(np.eye(6)[None] + G)
    return np.swapaxes(Ci, 1, 2) @ Ph @ Ci


def jacobi_blocks(S):
    nb = S.shape[0] // 6
    return np.stack([np.linalg.inv(S[6 * i:6 * i + 6, 6 * i:6 * i + 6]) for i in range(nb)])


def apply_blocks(P, r):
    nb = P.shape[0]
    return np.einsum("bij,bj->bi", P, r.reshape(nb, 6)).reshape(-1)


def pcg(S, b, P, tol=1e-8, max_iters=10000):
    """Preconditioned conjugate gradients for S x = b from x = 0 with
    M^{-1} = blockdiag(P). Returns (x, iterations, relative residual norms)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_blocks(P, r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0.0:
        return x, 0, hist
    for k in range(1, max_iters + 1):
        q = S @ p
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] <= tol:
            return x, k, hist
        z = apply_blocks(P, r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iters, hist
