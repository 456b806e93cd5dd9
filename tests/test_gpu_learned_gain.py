"""What the trained interpolation network gains over the method without it.

Networks are trained on the GPU (the library's own kernels) on harvested
BAMG^2 corrections of a few tandem chains, then one-cycle setups with the
network (learned="use", exact-LS fallback at twice the LS objective) are
compared with plain BAMG on held-out chains of other sizes and rates.

The outcome on the hardest held-out chain depends on the training seed
(the network's correction helps it a lot with some initialisations and
hurts it with others), so the test trains four seeds and asserts what
holds across them: the median total iteration count is below plain
BAMG's, every seed improves at least one chain, and no chain that plain
BAMG already solves in a few iterations gets more than one iteration
worse. Every solve must converge. The per-seed table is printed."""
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
    held_out = [(257, PAPER), (513, PAPER), (513, near_balanced(11)), (513, near_balanced(12)),
                (257, near_balanced(13)), (513, near_balanced(15))]
    chains = [chaingen.tandem(N, *rates) for N, rates in held_out]
    plain = [iterations(ch)[0] for ch in chains]
    print(f"held-out chains {[N for N, _ in held_out]}: BAMG {plain} total {sum(plain)}")
    totals = []
    for seed in (2024, 2025, 2026, 2027):
        net, losses = learned.train(X, T, M, seed=seed, epochs=120)
        assert losses[-1] < 0.5 * losses[0]
        runs = [iterations(ch, learned="use", mlp=net) for ch in chains]
        lrn = [it for it, _ in runs]
        frac = sum(a for _, (a, b) in runs) / sum(a + b for _, (a, b) in runs)
        print(f"seed {seed}: learned {lrn} total {sum(lrn)} (MLP rows {100 * frac:.0f}%)")
        totals.append(sum(lrn))
        assert any(l < p for l, p in zip(lrn, plain))
        assert all(l <= p + 1 for l, p in zip(lrn, plain) if p <= 8)
    print(f"totals: BAMG {sum(plain)}, learned median {np.median(totals)} of {totals}")
    assert np.median(totals) < sum(plain)
