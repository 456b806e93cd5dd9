"""GPU tests of the batched entry points and the lanes-per-row autotuner:
a batch gives each chain exactly the result of its own setup and solve, a
bad chain fails alone, and autotuned hierarchies still match the oracle."""
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
def test_autotuned_hierarchy_matches_oracle(precision):
    ch = chaingen.delaunay_walk(3000, 12)
    kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
    h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, autotune=1, precision=precision, **kw))
    x, info = h.gmres(restart=20, tol=1e-13, maxit=400)
    xo, _ = oracle.Hierarchy(ch, oracle.options_for(ch, **kw)).gmres(m=20, tol=1e-14, maxit=400)
    assert info.converged
    xs = x.cpu().numpy()
    assert np.abs(xs - xo).sum() / np.abs(xo).sum() < 1e-10
