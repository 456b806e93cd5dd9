"""What the trained interpolation network gains over the method without it.

Networks are trained on the GPU (the library's own kernels) on harvested
BAMG^2 corrections of a few tandem chains, then one-cycle setups with the
network (learned="use", exact-LS fallback at twice the LS objective) are
compared with plain BAMG on held-out chains of other sizes and rates.

Measured behaviour: on the chains plain BAMG already solves in 6-8
iterations the network changes the count by at most one; on the
moderately hard chain (12 iterations) every trained network brings it to
7; on the hardest chain (29 iterations) the outcome depends on the
training seed and on rounding-level details of the harvested data (about
half of the networks take it to 17-21 iterations, the others to 32-58).
The test trains four seeds, prints the table, and asserts what holds for
every network: each improves at least one held-out chain, none makes an
easy chain (<= 8 iterations) more than one iteration slower, and every
solve converges. The learned solves run with the library's iteration
fallback (learned_max_iters two past plain BAMG's count): a chain that is
still unconverged then is set up again with the exact fits and finished
from its iterate, so it ends within that budget plus a plain solve."""
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
    stats = h.learned_stats() if kw.get("learned") == "use" else None
    _, info = h.gmres(restart=20, tol=1e-10, maxit=300)
    h.close()
    assert info.converged
    return info.iterations, stats, info.mlp_fallback


def test_learned_interpolation_gain_per_network():
    from paper_1402_4005_amd import learned
    train_set = [chaingen.tandem(N, *r) for N, r in
                 [(33, PAPER), (65, PAPER), (129, PAPER), (65, near_balanced(1)),
                  (129, near_balanced(2)), (129, near_balanced(3)), (257, near_balanced(4))]]
    X, T, M = learned.harvest(train_set, **KW)
    held_out = [(257, PAPER), (513, PAPER), (513, near_balanced(11)), (513, near_balanced(12)),
                (257, near_balanced(13)), (513, near_balanced(15))]
    chains = [chaingen.tandem(N, *rates) for N, rates in held_out]
    plain = [iterations(ch)[0] for ch in chains]
    print(f"held-out chains {[N for N, _ in held_out]}: BAMG {plain} total {sum(plain)}")
    totals = []
    for seed in (2024, 2025, 2026, 2027):
        net, losses = learned.train(X, T, M, seed=seed, epochs=120)
        assert losses[-1] < 0.5 * losses[0]
        # iteration fallback two iterations past plain BAMG's count
        runs = [iterations(ch, learned="use", mlp=net, learned_max_iters=p + 2)
                for ch, p in zip(chains, plain)]
        lrn = [it for it, _, _ in runs]
        fbs = [f for _, _, f in runs]
        frac = sum(a for _, (a, b), _ in runs) / sum(a + b for _, (a, b), _ in runs)
        print(f"seed {seed}: learned {lrn} total {sum(lrn)} (MLP rows {100 * frac:.0f}%, "
              f"iteration fallbacks {fbs})")
        totals.append(sum(lrn))
        assert any(l < p for l, p in zip(lrn, plain))
        assert all(l <= p + 1 for l, p in zip(lrn, plain) if p <= 8)
        # a chain the network slows down is caught by the fallback: it never
        # takes more than the budget plus a plain solve from a better start
        for l, p, f in zip(lrn, plain, fbs):
            assert l <= p + 2 if not f else l <= 2 * p + 2, (l, p, f)
    print(f"totals: BAMG {sum(plain)}, learned {totals} (median {np.median(totals)})")
