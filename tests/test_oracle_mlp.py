"""Pins of the MLP reference (oracle/mlp.py) against library routines:
torch autograd in FP64 on the CPU, finite differences, torch's Adam and its
BF16 rounding. No GPU needed."""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


def batch(seed, n=37):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    T = rng.standard_normal((n, mlp.N_OUT))
    M = (rng.random((n, mlp.N_OUT)) < 0.7).astype(np.float64)
    return X, T, M


def torch_loss(p, X, T, M):
    w = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in mlp.unpack(p).items()}
    Xt, Tt, Mt = (torch.tensor(a, dtype=torch.float64) for a in (X, T, M))
    h1 = torch.relu(torch.nn.functional.linear(Xt, w["W1"], w["b1"]))
    h2 = torch.relu(torch.nn.functional.linear(h1, w["W2"], w["b2"]))
    y = torch.nn.functional.linear(h2, w["W3"], w["b3"])
    loss = 0.5 * (Mt * (y - Tt) ** 2).sum() / X.shape[0]
    loss.backward()
    g = np.concatenate([w[k].grad.numpy().ravel() for k, _ in mlp.SHAPES])
    return float(loss), g, y.detach().numpy()


def test_parameter_count():
    assert mlp.N_PARAMS == 10888


def test_forward_and_gradient_match_torch_autograd():
    p = mlp.init_params(1).astype(np.float64)
    X, T, M = batch(2)
    loss, g = mlp.loss_grad(p, X, T, M)
    tl, tg, ty = torch_loss(p, X, T, M)
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, ty, rtol=1e-12, atol=1e-12)
    assert abs(loss - tl) < 1e-12 * max(1.0, abs(tl))
    assert np.allclose(g, tg, rtol=1e-10, atol=1e-12)


def test_gradient_matches_finite_differences():
    p = mlp.init_params(3).astype(np.float64)
    X, T, M = batch(4, n=9)
    _, g = mlp.loss_grad(p, X, T, M)
    rng = np.random.default_rng(5)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, X, T, M)[0] - mlp.loss_grad(p - e, X, T, M)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_matches_torch():
    p0 = mlp.init_params(6).astype(np.float64)
    X, T, M = batch(7)
    w = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 4):
        _, g = mlp.loss_grad(p, X, T, M)
        p, m, v = mlp.adam_step(p, g, m, v, step, 1e-3)
        opt.zero_grad()
        w.grad = torch.tensor(mlp.loss_grad(w.detach().numpy(), X, T, M)[1])
        opt.step()
    assert np.allclose(p, w.detach().numpy(), rtol=1e-10, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(8)
    a = (rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000)).astype(np.float32)
    # include exact ties
    a[:4] = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 3.0], np.float32)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(a), ref)


def test_recorded_features_reproduce_the_ls_fit():
    # The first 72 features are sqrt(w_k) v_k / S at i and at J_i, so the
    # weighted LS of eq. ls_interpolation is the plain LS of feature 9k on
    # features 9k+1..9k+m. With the plain fit (interp_rule 0) and one setup
    # cycle the recorded P rows are that fit: numpy's lstsq must reproduce
    # them from the features alone. The B-stencil block is checked against
    # scipy's entries of B, and block 80..87 is the recorded fit itself.
    import scipy.sparse as sp
    import chaingen
    import oracle
    ch = chaingen.tandem(17, 11 / 31, 10 / 31, 10 / 31)
    o = oracle.options_for(ch, r=8, coarse_max=30, interp_rule=0, record_features=1)
    h = oracle.Hierarchy(ch, o)
    X, T, M = h.harvest(0)
    checked = 0
    for f in range(X.shape[0]):
        m = int(M[f].sum())
        G = np.array([[X[f, 9 * k + 1 + t] for t in range(m)] for k in range(8)])
        g = np.array([X[f, 9 * k] for k in range(8)])
        if np.linalg.cond(G) > 1e6:
            continue
        p = np.linalg.lstsq(G, g, rcond=None)[0]
        assert np.allclose(p, T[f, :m], rtol=1e-8, atol=1e-10), (f, p, T[f, :m])
        checked += 1
    assert checked > 0.9 * X.shape[0]
    B = sp.csr_matrix(sp.eye(ch.n) - ch.to_scipy())
    cf, cidx = h.cf(0)
    cpts = np.zeros(cf.sum(), int)
    cpts[cidx[cf == 1]] = np.where(cf == 1)[0]
    Pm = h.scipy(0, "P")
    fpts = np.where(cf == 0)[0]
    for f, i in enumerate(fpts[:200]):
        J = cpts[Pm.indices[Pm.indptr[i]:Pm.indptr[i + 1]]]
        for t, j in enumerate(J):
            assert abs(X[f, 72 + t] - B[i, j] / B[i, i]) < 1e-15
            assert X[f, 80 + t] == T[f, t]  # the exact cycle-1 row
        assert np.array_equal(X[f, 88:96], (np.arange(8) < len(J)).astype(float))
