"""Pins of the oracle's compatible-relaxation coarsening (reading R-CR of
the algebraic coarsening the paper cites, Section 7), CPU only:

* with a rate target no round can miss, only the completion step runs, and
  the split is the greedy maximal independent set of R-MIS (pinned itself
  against Luby rounds in test_oracle.py);
* the first round's F-relaxation rate equals the one formed from the dense
  iteration matrix S = I - omega D^-1 B (matrix powers, not sweeps);
* one and two full rounds (relaxation, candidates, the independent set in
  decreasing (candidate neighbours, priority) order, the completion) equal
  a separate numpy / Python implementation of the reading;
* on default parameters every F point has a coarse neighbour, the rate
  falls below the target, and the hierarchy solves a random walk to its
  closed-form stationary vector pi_i ~ deg(i).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import chaingen
import oracle

SEED = 14024009
OMEGA = 0.7


def operator_and_graph(ch):
    A = ch.to_scipy().tocsr()
    B = (sp.identity(ch.n, format="csr") - A).tocsr()
    B.sort_indices()
    G = (abs(B) + abs(B.T)).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return B, G


def priorities(n, level):
    return [int(oracle.philox4x64([i, level, 2, 0], [SEED, 0])[0]) for i in range(n)]


def start_error(pr):
    return np.array([0.5 + (p >> 11) * 2.0 ** -53 for p in pr])


def greedy(G, order_keys, part, cf):
    """Visit the participating vertices by decreasing (key, index); an
    undecided one joins C and its participating neighbours leave."""
    idx = [i for i in range(len(part)) if part[i]]
    idx.sort(key=lambda i: (order_keys[i], i), reverse=True)
    state = {i: 0 for i in idx}
    for v in idx:
        if state[v]:
            continue
        state[v] = 1
        cf[v] = 1
        for u in G.indices[G.indptr[v]:G.indptr[v + 1]]:
            if part[u] and state.get(u, 1) == 0:
                state[u] = 2


def reference_cr(B, G, level, theta, beta, sweeps, rounds):
    """R-CR written with dense matrices: per round e = S_F^k e0 with S_F =
    I - omega D^-1 B on the F rows and zero C entries."""
    n = B.shape[0]
    Bd = B.toarray()
    dinv = 1.0 / np.diag(Bd)
    pr = priorities(n, level)
    e0 = start_error(pr)
    cf = np.zeros(n, np.int64)
    rates, margins = [], []
    for _ in range(rounds):
        F = cf == 0
        S = np.eye(n) - OMEGA * dinv[:, None] * Bd
        S[~F, :] = 0.0
        S[:, ~F] = 0.0
        e = np.where(F, e0, 0.0)
        prev = e
        for _ in range(sweeps):
            prev, e = e, S @ e
        rate = np.linalg.norm(e) / np.linalg.norm(prev)
        rates.append(rate)
        if rate <= theta:
            break
        emax = np.abs(e[F]).max()
        part = F & (np.abs(e) >= beta * emax)
        margins.append(np.min(np.abs(np.abs(e[F]) - beta * emax)) / emax)
        w = np.array([part[G.indices[G.indptr[i]:G.indptr[i + 1]]].sum() for i in range(n)])
        keys = [(int(w[i]) << 48) + (pr[i] >> 16) for i in range(n)]
        greedy(G, keys, part, cf)
    part = np.array([cf[i] == 0 and not cf[G.indices[G.indptr[i]:G.indptr[i + 1]]].any()
                     for i in range(n)])
    greedy(G, pr, part, cf)
    return cf, np.array(rates), margins


CHAINS = [
    ("delaunay400", lambda: chaingen.delaunay_walk(400, 31)),
    ("hub300", lambda: chaingen.hub_walk(300, 3, 40, 7)),
]


@pytest.mark.parametrize("name,make", CHAINS, ids=[c[0] for c in CHAINS])
def test_cr_without_rounds_is_the_greedy_mis(name, make):
    B, G = operator_and_graph(make())
    cf, rates = oracle.cr(B, G, SEED, 1, theta=1e300)
    assert len(rates) == 1  # the first round's rate is always below the target
    assert np.array_equal(cf, oracle.mis(G.indptr, G.indices, SEED, 1))


@pytest.mark.parametrize("name,make", CHAINS, ids=[c[0] for c in CHAINS])
def test_cr_first_rate_from_the_iteration_matrix(name, make):
    B, G = operator_and_graph(make())
    _, rates = oracle.cr(B, G, SEED, 0, theta=1e300, sweeps=5)
    _, want, _ = reference_cr(B, G, 0, 1e300, 0.7, 5, 1)
    assert abs(rates[0] - want[0]) <= 1e-13 * want[0]


@pytest.mark.parametrize("rounds", [1, 2])
@pytest.mark.parametrize("name,make", CHAINS, ids=[c[0] for c in CHAINS])
def test_cr_rounds_match_dense_reimplementation(name, make, rounds):
    B, G = operator_and_graph(make())
    cf, rates = oracle.cr(B, G, SEED, 2, theta=-1.0, beta=0.7, sweeps=4, rounds=rounds)
    want, want_rates, margins = reference_cr(B, G, 2, -1.0, 0.7, 4, rounds)
    # no F point within rounding distance of the candidate threshold, so the
    # two summation orders must agree on every decision
    assert min(margins) > 1e-9
    assert len(rates) == rounds
    assert np.allclose(rates, want_rates, rtol=1e-12, atol=0)
    assert np.array_equal(cf, want)
    assert cf.sum() > oracle.mis(G.indptr, G.indices, SEED, 2).sum() // 2


def test_cr_defaults_cover_and_converge():
    ch = chaingen.delaunay_walk(2000, 33)
    B, G = operator_and_graph(ch)
    cf, rates = oracle.cr(B, G, SEED, 0)
    for i in np.flatnonzero(cf == 0):
        assert cf[G.indices[G.indptr[i]:G.indptr[i + 1]]].any(), i
    assert len(rates) < 10 and rates[-1] <= 0.8 < rates[0]
    assert np.all(np.diff(rates) < 0)


def test_cr_hierarchy_solves_random_walk_to_closed_form():
    ch = chaingen.delaunay_walk(1500, 34)
    kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99,
              coarsening="cr")
    h = oracle.Hierarchy(ch, oracle.options_for(ch, **kw))
    assert h.levels >= 3
    oc, og = h.complexity()
    assert og < 1.4 and oc < 1.7
    x, info = h.gmres(m=20, tol=1e-12, maxit=200)
    assert info.converged
    A = ch.to_scipy()
    deg = np.diff(A.tocsc().indptr).astype(float)  # out-degree of each state
    pi = deg / deg.sum()
    assert np.abs(x - pi).sum() < 1e-9
