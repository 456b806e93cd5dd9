"""GPU tests of the learned interpolation weights (an addition to the paper):
the MLP kernels against the FP64 reference in oracle/mlp.py, the recorded
features against the oracle's, and the learned setup's choice between the
MLP row and the exact LS row."""
import numpy as np
import pytest

import chaingen
import oracle
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

bamg = pytest.importorskip("paper_1402_4005_amd")


def data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 96)).astype(np.float32)
    T = rng.standard_normal((n, 8)).astype(np.float32)
    M = (rng.random((n, 8)) < 0.6).astype(np.float32)
    return X, T, M


def cuda(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def test_forward_fp32_matches_reference():
    p = bamg.mlp_init_params(1)
    X, _, _ = data(2, 1000)
    net = bamg.MLP(p)
    (Xd,) = cuda(X)
    y = net.forward(Xd, mode=0).cpu().numpy()
    yr, _ = ref.forward(p, X)
    assert np.abs(y - yr).max() < 1e-5 * max(1.0, np.abs(yr).max())


def test_forward_mfma_bf16_matches_reference():
    # BF16 weights, inputs and hidden activations, FP32 accumulation on MFMA;
    # the reference rounds at the same points and accumulates exactly. A
    # hidden value on a BF16 rounding boundary may round the other way
    # (one BF16 ulp, 2^-8 relative), so the bound is a few such ulps.
    p = bamg.mlp_init_params(3)
    X, _, _ = data(4, 1003)  # ragged: not a multiple of 16 or 64
    net = bamg.MLP(p)
    (Xd,) = cuda(X)
    y = net.forward(Xd, mode=1).cpu().numpy()
    yr, _ = ref.forward(p, X, bf16=True)
    scale = np.abs(yr).max()
    err = np.abs(y - yr)
    assert err.max() < 2e-2 * scale, err.max() / scale
    assert np.median(err) < 1e-4 * scale
    # and close to the FP32 network
    y32, _ = ref.forward(p, X)
    assert np.abs(y - y32).max() < 5e-2 * np.abs(y32).max()


def test_gradient_matches_reference():
    p = bamg.mlp_init_params(5)
    X, T, M = data(6, 2048)
    net = bamg.MLP(p)
    loss, g = net.loss_grad(*cuda(X, T, M))
    g = g.cpu().numpy()
    lr, gr = ref.loss_grad(p, X, T, M)
    assert abs(loss - lr) < 1e-5 * lr
    assert np.abs(g - gr).max() < 1e-4 * np.abs(gr).max()
    assert np.linalg.norm(g - gr) < 1e-5 * np.linalg.norm(gr)


def test_adam_step_matches_reference_and_training_converges():
    p = bamg.mlp_init_params(7)
    X, T, M = data(8, 512)
    net = bamg.MLP(p)
    Xd, Td, Md = cuda(X, T, M)
    net.train(Xd, Td, Md, batch=512, epochs=1, lr=1e-3)
    _, g = ref.loss_grad(p, X, T, M)
    pr, _, _ = ref.adam_step(p.astype(np.float64), g, 0.0, 0.0, 1, 1e-3)
    pg = net.params()
    assert np.abs(pg - pr).max() < 1e-6 + 1e-5 * np.abs(pr).max()
    # a target the network can represent: a fixed teacher network
    teacher = bamg.mlp_init_params(9)
    Xt, _, _ = data(10, 4096)
    Tt = ref.forward(teacher, Xt)[0].astype(np.float32)
    Mt = np.ones_like(Tt)
    student = bamg.MLP(bamg.mlp_init_params(11))
    losses = student.train(*cuda(Xt, Tt, Mt), batch=256, epochs=30, lr=2e-3)
    assert losses[-1] < 0.25 * losses[0], losses
    assert losses[-1] < losses[len(losses) // 2], losses


CHAINS = [
    ("tandem17", lambda: chaingen.tandem(17, 11 / 31, 10 / 31, 10 / 31), dict(coarse_max=30)),
    ("delaunay1500", lambda: chaingen.delaunay_walk(1500, 3),
     dict(max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)),
]


@pytest.mark.parametrize("name,make,kw", CHAINS, ids=[c[0] for c in CHAINS])
def test_harvest_matches_oracle(name, make, kw):
    ch = make()
    ho = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, setup_cycles=2, record_features=1, **kw))
    hg = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, r=8, setup_cycles=2,
                                                        learned="record", **kw))
    assert ho.levels == hg.levels
    for l in range(ho.levels - 1):
        Xo, To, Mo = ho.harvest(l)
        Xg, Tg, Mg = (a.cpu().numpy() for a in hg.harvest(l))
        assert Xg.shape == Xo.shape
        assert np.array_equal(Mg, Mo)
        assert np.abs(Xg - Xo).max() < 1e-6, (l, np.abs(Xg - Xo).max())
        assert np.abs(Tg - To).max() < 1e-6 * max(1.0, np.abs(To).max()), l


def test_learned_rows_follow_the_objective_rule():
    # Level 0's cycle-1 features and LS rows are the same with and without
    # the network (nothing before the first fit depends on it). Every F row
    # of P in learned mode must be the LS row plus the MFMA correction when
    # its LS objective, computable from the features, is within twice the
    # exact fit's, and the exact row otherwise; x must still be the
    # stationary vector.
    import torch
    ch = chaingen.tandem(33, 11 / 31, 10 / 31, 10 / 31)
    kw = dict(r=8, coarse_max=300, nu_setup=3)
    rec = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, learned="record", **kw))
    X, T_ls, M = (a.cpu().numpy() for a in rec.harvest(0))
    # a network trained towards small random corrections of the LS rows, so
    # that some rows pass the objective test and some do not
    assert np.array_equal(X[:, 80:88], T_ls)
    rng = np.random.default_rng(13)
    Tc = (0.05 * rng.standard_normal(T_ls.shape) * M).astype(np.float32)
    net = bamg.MLP(bamg.mlp_init_params(12))
    Xd, Td, Md = (torch.from_numpy(a).cuda() for a in (X, Tc, M))
    net.train(Xd, Td, Md, batch=256, epochs=20, lr=2e-3)
    Y = T_ls + net.forward(Xd, mode=1).cpu().numpy() * M
    use = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, learned="use", mlp=net, **kw))
    Pm = use.scipy(0, "P")
    cf, _ = use.cf(0)
    fpts = np.where(cf == 0)[0]
    n_mlp = n_ls = 0
    for f, i in enumerate(fpts):
        m = int(M[f].sum())
        row = Pm.data[Pm.indptr[i]:Pm.indptr[i] + m]
        g = X[f, 0:72:9].astype(np.float64)
        G = np.stack([X[f, 1 + t:72:9] for t in range(m)], 1).astype(np.float64)
        jm = ((g - G @ Y[f, :m]) ** 2).sum()
        jl = ((g - G @ T_ls[f, :m]) ** 2).sum()
        if abs(jm - 2 * jl) <= 1e-4 * (jm + 2 * jl):
            continue  # too close to the threshold to decide in FP32 features
        info = (f, i, m, row, Y[f, :m], T_ls[f, :m], jm, jl)
        if jm <= 2 * jl:
            assert np.allclose(row, Y[f, :m], rtol=0, atol=2e-6), info
            n_mlp += 1
        else:
            assert np.allclose(row, T_ls[f, :m], rtol=1e-6, atol=1e-7), info  # FP32 harvest
            n_ls += 1
    assert n_mlp > 0
    a, b = use.learned_stats()
    assert a + b == sum(int((use.cf(l)[0] == 0).sum()) for l in range(use.levels - 1))
    x, info = use.gmres(restart=20, tol=1e-14, maxit=400)
    assert (info.mlp_rows, info.ls_fallbacks) == (a, b)
    xo, _ = oracle.Hierarchy(ch, oracle.options_for(ch, **kw)).gmres(m=20, tol=1e-14, maxit=400)
    assert info.converged
    xs = x.cpu().numpy()
    assert np.abs(xs - xo).sum() / np.abs(xo).sum() < 1e-10


def test_learned_iteration_fallback():
    """The learned form's GMRES-iteration fallback: with learned_max_iters = 1
    a learned hierarchy that has not converged after one iteration is
    replaced by the exact-LS one (same options, learned off) and GMRES goes on
    from its iterate. The solve converges, reports the fallback, counts both
    parts, and ends at the plain BAMG solution (1e-10)."""
    import torch
    ch = chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31)
    kw = dict(r=8, max_interp=4, coarse_max=300, nu_setup=8)
    net = bamg.MLP(bamg.mlp_init_params(3))  # untrained: poor corrections
    hl = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, learned="use", mlp=net,
                                                        learned_max_iters=1, **kw))
    xl, il = hl.gmres(restart=20, tol=1e-12, maxit=300)
    hp = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, **kw))
    xp, ip = hp.gmres(restart=20, tol=1e-12, maxit=300)
    torch.cuda.synchronize()
    assert il.converged and ip.converged
    assert il.mlp_fallback == 1
    assert il.iterations >= 2
    assert il.t_setup_ms > 0
    assert hl.learned_stats() == (0, 0)  # the hierarchy now is the exact-LS one
    assert (il.mlp_rows, il.ls_fallbacks) == (0, 0)
    xl, xp = xl.cpu().numpy(), xp.cpu().numpy()
    assert np.abs(xl - xp).sum() / np.abs(xp).sum() < 1e-10
    # without the cap there is no fallback
    hn = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, learned="use", mlp=net, **kw))
    _, inn = hn.gmres(restart=20, tol=1e-12, maxit=300)
    assert inn.mlp_fallback == 0
    net.close()
