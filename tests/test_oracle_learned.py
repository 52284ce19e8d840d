"""Pins of the learned-preconditioner oracle (oracle/learned.py) against
closed forms, independent dense algebra, Monte Carlo expectations, finite
differences and textbook properties of conjugate gradients."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import learned as LP


def random_spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    w = np.geomspace(1.0, cond, n)
    return (Q * w) @ Q.T


def test_whitening_gives_identity_blocks():
    S = random_spd(36, 1)
    C, Ci, G = LP.block_whitening(S)
    for i in range(6):
        np.testing.assert_allclose(Ci[i] @ S[6 * i:6 * i + 6, 6 * i:6 * i + 6] @ Ci[i].T, np.eye(6), atol=1e-10)
    Sd = sl.block_diag(*[S[6 * i:6 * i + 6, 6 * i:6 * i + 6] for i in range(6)])
    _, _, G0 = LP.block_whitening(Sd)
    assert np.abs(G0).max() == 0.0


def test_coupling_is_diagonal_block_of_whitened_square():
    """(S^ S^)_ii = I + G_i with S^ = D S D^T formed densely."""
    S = random_spd(42, 2)
    _, Ci, G = LP.block_whitening(S)
    D = sl.block_diag(*[np.linalg.inv(np.linalg.cholesky(S[6 * i:6 * i + 6, 6 * i:6 * i + 6])) for i in range(7)])
    Sh = D @ S @ D.T
    Sq = Sh @ Sh
    for i in range(7):
        np.testing.assert_allclose(Sq[6 * i:6 * i + 6, 6 * i:6 * i + 6] - np.eye(6), G[i], rtol=1e-9, atol=1e-9)


def test_features_layout():
    G = np.zeros((1, 6, 6))
    G[0] = np.diag(np.arange(1.0, 7.0))
    G[0, 0, 5] = G[0, 5, 0] = 0.5
    x = LP.features(G)[0]
    tr = 21.0
    assert x.shape == (22,)
    assert x[0] == pytest.approx(1.0 / (1 + tr)) and x[5] == pytest.approx(0.5 / (1 + tr))
    assert x[20] == pytest.approx(6.0 / (1 + tr)) and x[21] == pytest.approx(np.log(1 + tr))


def test_loss_is_expected_block_residual():
    """l_i = E ||P^ (S^ z)_i - z_i||^2 over z ~ N(0, I), by Monte Carlo."""
    S = random_spd(30, 3, cond=50.0)
    _, Ci, G = LP.block_whitening(S)
    D = sl.block_diag(*Ci)
    Sh = D @ S @ D.T
    rng = np.random.default_rng(4)
    Y = 0.3 * rng.normal(size=(5, 21))
    loss, _ = LP.block_loss(Y, G)
    L = LP.factor_from_output(Y)
    Z = rng.normal(size=(30, 200000))
    R = Sh @ Z
    for i in range(5):
        Ph = L[i] @ L[i].T
        e = Ph @ R[6 * i:6 * i + 6] - Z[6 * i:6 * i + 6]
        mc = np.mean(np.sum(e * e, axis=0))
        assert mc == pytest.approx(loss[i], rel=2e-2)


def test_loss_minimizer_and_identity():
    S = random_spd(24, 5)
    _, _, G = LP.block_whitening(S)
    # zero output: P^ = I, loss = tr(G)
    loss0, _ = LP.block_loss(np.zeros((4, 21)), G)
    np.testing.assert_allclose(loss0, np.trace(G, axis1=1, axis2=2), rtol=1e-12)
    # output whose P^ is (I + G)^{-1}: zero gradient, loss 6 - tr((I + G)^{-1})
    Y = np.zeros((4, 21))
    for i in range(4):
        Lm = np.linalg.cholesky(np.linalg.inv(np.eye(6) + G[i]))
        for k, (r, c) in enumerate(LP.TRI):
            Y[i, k] = np.log(Lm[r, c]) if r == c else Lm[r, c]
    loss, dY = LP.block_loss(Y, G)
    assert np.abs(dY).max() < 1e-10
    np.testing.assert_allclose(loss, 6.0 - np.trace(np.linalg.inv(np.eye(6)[None] + G), axis1=1, axis2=2),
                               rtol=1e-10)


def test_optimal_blocks_are_the_loss_minimizer():
    """optimal_blocks: on a block-diagonal system (G = 0) it is block Jacobi;
    in general its whitened blocks are the stationary point of the block loss
    (dense inverse of I + G, computed here from the densely whitened S^2), and
    no perturbed output has a lower loss."""
    S = random_spd(24, 9)
    Sd = np.zeros_like(S)
    for i in range(4):
        Sd[6 * i:6 * i + 6, 6 * i:6 * i + 6] = S[6 * i:6 * i + 6, 6 * i:6 * i + 6]
    np.testing.assert_allclose(LP.optimal_blocks(Sd), LP.jacobi_blocks(Sd), rtol=1e-10, atol=1e-14)
    C, Ci, G = LP.block_whitening(S)
    D = sl.block_diag(*Ci)
    Sh = D @ S @ D.T
    Sh2 = Sh @ Sh
    P = LP.optimal_blocks(S)
    for i in range(4):
        want = np.linalg.inv(Sh2[6 * i:6 * i + 6, 6 * i:6 * i + 6])      # (I + G_i)^{-1} = ((S^ S^)_ii)^{-1}
        np.testing.assert_allclose(C[i].T @ P[i] @ C[i], want, rtol=1e-9, atol=1e-12)
    rng = np.random.default_rng(3)
    Y = np.zeros((4, 21))
    for i in range(4):
        Lm = np.linalg.cholesky(C[i].T @ P[i] @ C[i])
        for k, (r, c) in enumerate(LP.TRI):
            Y[i, k] = np.log(Lm[r, c]) if r == c else Lm[r, c]
    best, _ = LP.block_loss(Y, G)
    for _ in range(20):
        worse, _ = LP.block_loss(Y + 1e-3 * rng.normal(size=Y.shape), G)
        assert np.all(worse >= best - 1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(6)
    p = LP.init_params(7)
    p["W3"] = 0.05 * rng.normal(size=p["W3"].shape)
    p["b3"] = 0.05 * rng.normal(size=21)
    p["b1"] = 0.1 * rng.normal(size=256)
    G = np.stack([0.5 * (lambda a: a @ a.T)(rng.normal(size=(6, 6))) for _ in range(9)])
    X = LP.features(G)
    loss, g = LP.loss_and_grads(p, X, G)
    h = 1e-6
    for name, shape in LP.PARAM_SHAPES:
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in shape)
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            lp, _ = LP.loss_and_grads(q, X, G)
            q[name][idx] -= 2 * h
            lm, _ = LP.loss_and_grads(q, X, G)
            fd = (lp - lm) / (2 * h)
            assert g[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, idx)


def test_pack_roundtrip_and_size():
    p = LP.init_params(1)
    v = LP.pack(p)
    assert v.size == LP.N_PARAMS == 22 * 256 + 256 + 256 * 256 + 256 + 256 * 21 + 21
    q = LP.unpack(v)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])


def test_zero_network_is_block_jacobi():
    S = random_spd(36, 8)
    np.testing.assert_allclose(LP.learned_blocks(LP.init_params(2), S), LP.jacobi_blocks(S), rtol=1e-10,
                               atol=1e-12)


def test_pcg_solves_spd_system():
    S = random_spd(60, 9, cond=1e4)
    b = np.random.default_rng(10).normal(size=60)
    x, k, hist = LP.pcg(S, b, LP.jacobi_blocks(S), tol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(S, b), rtol=1e-8, atol=1e-10 * np.abs(x).max())
    assert hist[-1] <= 1e-12 and k <= 200


def test_pcg_exact_block_preconditioner_takes_one_step():
    S = sl.block_diag(*[random_spd(6, 20 + i) for i in range(5)])
    b = np.random.default_rng(11).normal(size=30)
    x, k, _ = LP.pcg(S, b, LP.jacobi_blocks(S), tol=1e-12)
    assert k == 1
    np.testing.assert_allclose(S @ x, b, rtol=1e-12, atol=1e-12)


def test_cg_terminates_in_number_of_distinct_eigenvalues():
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.normal(size=(36, 36)))
    w = np.repeat([1.0, 4.0, 9.0], 12)
    S = (Q * w) @ Q.T
    b = rng.normal(size=36)
    _, k, _ = LP.pcg(S, b, np.stack([np.eye(6)] * 6), tol=1e-10)
    assert k <= 3
