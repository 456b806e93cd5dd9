"""GPU tests of the batched entry points and the lanes-per-row autotuner:
a batch gives each chain exactly the result of its own setup and solve, a
bad chain fails alone, and autotuned hierarchies still match the oracle.

The batched solve runs in one persistent launch by default (a workgroup per
chain); its results must equal those of the per-chain solve bit for bit, on
the same handles and on hierarchies set up separately, for every form it
takes (FP64 and mixed precision, Jacobi and Kaczmarz, fused or unfused last
level, no preconditioner, unconverged chains), and chains it does not take
(W-cycles) must go through the per-chain solve unchanged."""
import numpy as np
import pytest

import chaingen
import oracle

pytestmark = pytest.mark.gpu

bamg = pytest.importorskip("paper_1402_4005_amd")


def members():
    out = [
        (chaingen.tandem(17, 11 / 31, 10 / 31, 10 / 31), dict(r=8, coarse_max=30)),
        (chaingen.delaunay_walk(3000, 21), dict(r=8, max_interp=3, nu_pre=5, nu_post=5,
                                                nu_setup=5, coarse_max=99)),
        (chaingen.tandem(33, 0.34, 0.33, 0.33), dict(r=8, coarse_max=300, nu_setup=5)),
        (chaingen.birth_death(257, 0.96), dict(r=8, max_interp=2, coarse_max=29)),
        (chaingen.delaunay_walk(1200, 22), dict(r=8, max_interp=3, nu_pre=5, nu_post=5,
                                                nu_setup=5, coarse_max=99)),
    ]
    return out


def test_batch_equals_individual_solves():
    import torch
    ms = members()
    chains = [c for c, _ in ms]
    opts = [bamg.options_for(c, **kw) for c, kw in ms]
    b = bamg.Batch(chains, opts, nstreams=3)
    xs, infos, sts = b.gmres(restart=20, tol=1e-12, maxit=300)
    torch.cuda.synchronize()
    for i, (c, kw) in enumerate(ms):
        assert sts[i] == 0 and infos[i].converged, (i, sts[i])
        h = bamg.Hierarchy.from_chain(c, bamg.options_for(c, **kw))
        x, info = h.gmres(restart=20, tol=1e-12, maxit=300)
        assert info.iterations == infos[i].iterations
        assert np.array_equal(x.cpu().numpy(), xs[i].cpu().numpy()), i


def test_batch_keeps_a_bad_chain_separate():
    ms = members()[:3]
    bad = chaingen.Chain(ms[0][0].to_scipy() * 1.01, ms[0][0].geom)
    chains = [ms[0][0], bad, ms[2][0]]
    opts = [bamg.options_for(c, **kw) for c, kw in (ms[0], ms[0], ms[2])]
    b = bamg.Batch(chains, opts, nstreams=2)
    assert b.status(0) == 0 and b.status(2) == 0
    assert b.status(1) == -2  # not column stochastic
    xs, infos, sts = b.gmres(restart=20, tol=1e-10, maxit=300)
    assert xs[1] is None and sts[1] == -2
    assert sts[0] == 0 and sts[2] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [3000, 20000])
def test_autotuned_hierarchy_matches_oracle(precision, n):
    """3,000 states: every level is too small to fill the chip, so none is
    timed (default lanes, 128 threads); 20,000: the finest level's lanes and
    workgroup size are timed. Either way x matches the oracle."""
    ch = chaingen.delaunay_walk(n, 12)
    kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
    h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, autotune=1, precision=precision, **kw))
    for l in range(h.levels - 1):
        rp, _, _ = h.csr(l, "B")
        avg = -(-int(rp[-1]) // (len(rp) - 1))
        dl = min(4, 1 << max(0, (avg - 1).bit_length()))
        if (len(rp) - 1) * dl < 256 * 256:
            assert (h.lanes(l), h.threads(l)) == (dl, 128), l
    x, info = h.gmres(restart=20, tol=1e-13, maxit=400)
    xo, _ = oracle.Hierarchy(ch, oracle.options_for(ch, **kw)).gmres(m=20, tol=1e-14, maxit=400)
    assert info.converged
    xs = x.cpu().numpy()
    assert np.abs(xs - xo).sum() / np.abs(xo).sum() < 1e-10


PLANAR = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
PAPER = (11 / 31, 10 / 31, 10 / 31)


def forms():
    """(chain, options keywords, maxit): one chain per form of the
    persistent solve."""
    return [
        (chaingen.tandem(17, *PAPER), dict(r=8, coarse_max=30), 300),
        (chaingen.delaunay_walk(3000, 21), PLANAR, 300),
        (chaingen.tandem(33, *PAPER), dict(r=8, coarse_max=300, nu_setup=5,
                                           precision="mixed"), 300),
        (chaingen.delaunay_walk(1200, 22), dict(PLANAR, smoother=1), 300),
        (chaingen.tandem(33, 0.34, 0.33, 0.33), dict(r=8, coarse_max=30, nu_setup=5,
                                                     fuse_last_level=0), 300),
        (chaingen.tandem(33, 0.34, 0.33, 0.33), dict(r=8, coarse_max=30, nu_setup=5), 300),
        (chaingen.delaunay_walk(6000, 23), dict(PLANAR, nu_pre=4, nu_post=3), 300),
        (chaingen.birth_death(257, 0.96), dict(r=8, max_interp=2, coarse_max=29), 300),
        (chaingen.tandem(65, *PAPER), dict(r=8, max_interp=4, coarse_max=300, nu_setup=8), 3),
        (chaingen.delaunay_walk(2000, 24), dict(PLANAR, cycle="none"), 40),
    ]


def solve_batch(ms, solver, restart=20, tol=1e-12):
    import torch
    chains = [c for c, _, _ in ms]
    opts = [bamg.options_for(c, **kw) for c, kw, _ in ms]
    # one maxit per call: chains that should stop early get their own batch
    outs = []
    for maxit in sorted(set(m for _, _, m in ms)):
        idx = [i for i, (_, _, m) in enumerate(ms) if m == maxit]
        sub = bamg.Batch([chains[i] for i in idx], [opts[i] for i in idx], nstreams=2)
        sub.set_solver(solver)
        xs, infos, sts = sub.gmres(restart=restart, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        outs += [(i, xs[k], infos[k], sts[k]) for k, i in enumerate(idx)]
        sub.close()
    return sorted(outs, key=lambda t: t[0])


@pytest.mark.parametrize("solver", ["persistent", "auto"])
def test_persistent_solve_equals_per_chain_solve(solver):
    """'persistent': every form in the launch; 'auto': the chains above 5000
    states (Delaunay 6000) on the streams while the others run in the launch."""
    ms = forms()
    per = solve_batch(ms, solver)
    ref = solve_batch(ms, "streams")
    for (i, x, inf, st), (_, xr, infr, str_) in zip(per, ref):
        assert st == str_, (i, st, str_)
        assert inf.iterations == infr.iterations, (i, inf.iterations, infr.iterations)
        assert inf.restarts == infr.restarts and inf.converged == infr.converged, i
        assert inf.rel_residual == infr.rel_residual, (i, inf.rel_residual, infr.rel_residual)
        assert inf.x_min == infr.x_min, i
        assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy()), i
    # what the forms exercise: converged chains, an unconverged one (maxit 3)
    assert sum(1 for _, _, inf, _ in per if inf.converged) >= 8
    assert per[8][3] == 1 and per[8][2].iterations == 3


def test_persistent_batch_matches_oracle_sample():
    """A 32-chain sample of the batched workload's families at small sizes
    (tandem queues 17^2..49^2 with random rates, Delaunay walks of 1k..4k
    points): each x within 1e-10 of the FP64 oracle (relative l1)."""
    import torch
    rng = np.random.default_rng(14024004)
    ms = []
    for k in range(32):
        if k % 2 == 0:
            N = int(rng.integers(17, 50))
            r = rng.uniform(0.25, 0.4, 3)
            ch = chaingen.tandem(N, *(r / r.sum()))
            kw = dict(r=8, max_interp=4, coarse_max=99, nu_setup=8)
        else:
            ch = chaingen.delaunay_walk(int(rng.integers(1000, 4000)), int(rng.integers(1 << 30)))
            kw = PLANAR
        ms.append((ch, kw))
    b = bamg.Batch([c for c, _ in ms], [bamg.options_for(c, **kw) for c, kw in ms], nstreams=4)
    xs, infos, sts = b.gmres(restart=20, tol=1e-13, maxit=400)
    torch.cuda.synchronize()
    for i, (c, kw) in enumerate(ms):
        assert sts[i] == 0 and infos[i].converged, (i, sts[i])
        xo, _ = oracle.Hierarchy(c, oracle.options_for(c, **kw)).gmres(m=20, tol=1e-14,
                                                                       maxit=400)
        x = xs[i].cpu().numpy()
        assert np.abs(x - xo).sum() / np.abs(xo).sum() < 1e-10, i
    b.close()


def test_w_cycle_chain_goes_through_per_chain_solve():
    import torch
    ms = [(chaingen.tandem(33, *PAPER), dict(r=8, coarse_max=30, cycle="W")),
          (chaingen.delaunay_walk(1500, 25), PLANAR)]
    b = bamg.Batch([c for c, _ in ms], [bamg.options_for(c, **kw) for c, kw in ms], nstreams=2)
    xs, infos, sts = b.gmres(restart=20, tol=1e-12, maxit=300)
    torch.cuda.synchronize()
    for i, (c, kw) in enumerate(ms):
        h = bamg.Hierarchy.from_chain(c, bamg.options_for(c, **kw))
        x, info = h.gmres(restart=20, tol=1e-12, maxit=300)
        assert sts[i] == 0 and info.iterations == infos[i].iterations, i
        assert np.array_equal(x.cpu().numpy(), xs[i].cpu().numpy()), i
    b.close()


@pytest.mark.parametrize("solver", ["persistent", "auto"])
def test_flexible_chains_solve_on_the_streams(solver):
    """Flexible-GMRES chains leave the persistent launch (it runs the
    left-preconditioned GMRES only) for the per-chain solve on the streams,
    whatever the solver asked for: the same bits as the streams alone."""
    ms = [(chaingen.tandem(33, *PAPER), dict(r=8, coarse_max=300, nu_setup=5, precision="mixed",
                                             flexible=1), 300),
          (chaingen.delaunay_walk(3000, 21), dict(PLANAR, flexible=1), 300),
          (chaingen.tandem(17, *PAPER), dict(r=8, coarse_max=30), 300)]
    per = solve_batch(ms, solver)
    ref = solve_batch(ms, "streams")
    for (i, x, inf, st), (_, xr, infr, str_) in zip(per, ref):
        assert st == 0 and str_ == 0 and inf.converged, (i, st, str_)
        assert inf.iterations == infr.iterations, i
        assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy()), i
