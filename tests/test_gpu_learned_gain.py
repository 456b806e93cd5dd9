"""What the trained interpolation network gains over the method without it.

The network is trained on the GPU (the library's own kernels) on harvested
BAMG^2 corrections of a few tandem chains, then a one-cycle setup with the
network (learned="use", exact-LS fallback at twice the LS objective) is
compared with plain BAMG on held-out chains of other sizes and rates. The
test prints the iteration table and asserts that the learned hierarchy
needs fewer GMRES iterations in total, with every solve converged."""
import numpy as np
import pytest

import chaingen

pytestmark = pytest.mark.gpu

bamg = pytest.importorskip("paper_1402_4005_amd")

PAPER = (11 / 31, 10 / 31, 10 / 31)
KW = dict(r=8, max_interp=4, coarse_max=300, nu_setup=8)


def near_balanced(seed):
    """Rates in [0.30, 0.36] before normalisation: both queues near balance."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.30, 0.36, 3)
    return tuple(r / r.sum())


def iterations(ch, **kw):
    h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, **KW, **kw), on_device=True)
    _, info = h.gmres(restart=20, tol=1e-10, maxit=300)
    stats = h.learned_stats() if kw.get("learned") == "use" else None
    h.close()
    assert info.converged
    return info.iterations, stats


def test_learned_interpolation_reduces_iterations():
    from paper_1402_4005_amd import learned
    train_set = [chaingen.tandem(N, *r) for N, r in
                 [(33, PAPER), (65, PAPER), (129, PAPER), (65, near_balanced(1)),
                  (129, near_balanced(2)), (129, near_balanced(3)), (257, near_balanced(4))]]
    X, T, M = learned.harvest(train_set, **KW)
    net, losses = learned.train(X, T, M, epochs=120)
    assert losses[-1] < 0.5 * losses[0]
    held_out = [(257, PAPER), (513, PAPER), (513, near_balanced(11)), (513, near_balanced(12)),
                (257, near_balanced(13)), (513, near_balanced(15))]
    rows = []
    for N, rates in held_out:
        ch = chaingen.tandem(N, *rates)
        plain, _ = iterations(ch)
        lrn, (n_mlp, n_ls) = iterations(ch, learned="use", mlp=net)
        rows.append((N, plain, lrn, n_mlp / (n_mlp + n_ls)))
    for N, plain, lrn, frac in rows:
        print(f"tandem {N}^2: BAMG {plain} iterations, learned {lrn} "
              f"(MLP rows {100 * frac:.0f}%)")
    total_plain = sum(r[1] for r in rows)
    total_learned = sum(r[2] for r in rows)
    print(f"total: BAMG {total_plain}, learned {total_learned}")
    assert total_learned < total_plain
