"""GPU tests of the variants beside plain FP64 Jacobi: the mixed-precision
form (FP32 setup and V-cycles, FP64 Krylov, residual, normalisation and
coarsest solve) and the Kaczmarz smoother. Both are compared with the FP64
CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

import chaingen
import oracle

pytestmark = pytest.mark.gpu

bamg = pytest.importorskip("paper_1402_4005_amd")


def rel_l1(x, y):
    return float(np.abs(x - y).sum() / np.abs(y).sum())


MIXED = [
    ("tandem65_random", lambda: chaingen.tandem(65, *chaingen.tandem_random_rates(14024003)),
     dict(r=8, coarse_max=99)),
    ("delaunay3000", lambda: chaingen.delaunay_walk(3000, 12),
     dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)),
]


@pytest.mark.parametrize("name,make,kw", MIXED, ids=[c[0] for c in MIXED])
def test_mixed_precision_structure_and_solution(name, make, kw):
    import torch
    ch = make()
    ho = oracle.Hierarchy(ch, oracle.options_for(ch, **kw))
    hm = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, precision="mixed", **kw))
    # integer structure does not depend on the precision
    assert ho.levels == hm.levels
    for l in range(ho.levels - 1):
        assert np.array_equal(ho.cf(l)[0], hm.cf(l)[0])
        for what in ("P", "Q"):
            assert np.array_equal(ho.csr(l, what)[1], hm.csr(l, what)[1])
    # FP32 transfer weights agree with the FP64 oracle to FP32 accuracy
    for l in range(ho.levels - 1):
        a, b = hm.csr(l, "P")[2], ho.csr(l, "P")[2]
        assert np.abs(a - b).max() < 2e-3 * max(1.0, np.abs(b).max())
    xo, io = ho.gmres(m=20, tol=1e-13, maxit=600)
    xm, im = hm.gmres(restart=20, tol=1e-13, maxit=600)
    torch.cuda.synchronize()
    assert im.converged, im.as_dict()
    # the FP64 true-residual test decides convergence, so x reaches FP64 accuracy
    assert rel_l1(xm.cpu().numpy(), xo) < 1e-10


def test_mixed_vcycle_f32_entry():
    import torch
    ch = chaingen.tandem(33, 11 / 31, 10 / 31, 10 / 31)
    kw = dict(r=6, max_levels=3, coarse_max=1)
    ho = oracle.Hierarchy(ch, oracle.options_for(ch, **kw))
    hm = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, precision="mixed", **kw))
    b = np.random.default_rng(3).standard_normal(ch.n)
    xo = ho.vcycle(b)
    x32 = hm.vcycle(torch.from_numpy(b.astype(np.float32)).cuda()).cpu().numpy()
    x64 = hm.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
    scale = np.abs(xo).max()
    assert np.abs(x32 - xo).max() < 1e-3 * scale
    assert np.abs(x64 - x32).max() < 1e-6 * scale


KACZ = [
    ("tandem14_2lev", lambda: chaingen.tandem(14, 11 / 31, 10 / 31, 10 / 31),
     dict(r=6, max_levels=2, coarse_max=1)),
    ("delaunay1500", lambda: chaingen.delaunay_walk(1500, 4),
     dict(r=8, max_interp=3, nu_pre=2, nu_post=2, nu_setup=2, coarse_max=99)),
]


@pytest.mark.parametrize("name,make,kw", KACZ, ids=[c[0] for c in KACZ])
def test_kaczmarz_matches_oracle(name, make, kw):
    import torch
    ch = make()
    ho = oracle.Hierarchy(ch, oracle.options_for(ch, smoother="kaczmarz", **kw))
    hg = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, smoother="kaczmarz", **kw))
    for l in range(1, ho.levels):
        a, b = hg.csr(l, "B")[2], ho.csr(l, "B")[2]
        assert np.abs(a - b).max() < 1e-8 * np.abs(b).max(), l
    b = np.random.default_rng(8).standard_normal(ch.n)
    xo = ho.vcycle(b)
    xg = hg.vcycle(torch.from_numpy(b).cuda()).cpu().numpy()
    assert np.abs(xg - xo).max() < 1e-8 * np.abs(xo).max()
    xo, io = ho.gmres(m=20, tol=1e-13, maxit=400)
    xg, ig = hg.gmres(restart=20, tol=1e-13, maxit=400)
    torch.cuda.synchronize()
    assert ig.converged and io.converged
    assert rel_l1(xg.cpu().numpy(), xo) < 1e-10


LAST = [
    ("delaunay20000", lambda: chaingen.delaunay_walk(20000, 5),
     dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)),
    ("tandem65_nu33", lambda: chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31),
     dict(r=8, coarse_max=30)),
    ("tandem65_nu21", lambda: chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31),
     dict(r=8, coarse_max=30, nu_pre=2, nu_post=1)),
    ("tandem65_nu04", lambda: chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31),
     dict(r=8, coarse_max=30, nu_pre=0, nu_post=4)),
    ("delaunay20000_mixed", lambda: chaingen.delaunay_walk(20000, 5),
     dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99, precision="mixed")),
]


@pytest.mark.parametrize("name,make,kw", LAST, ids=[c[0] for c in LAST])
def test_fused_last_level_matches_separate_steps(name, make, kw):
    """The one-workgroup cycle of the level above the coarsest (LDS-resident
    operator, transfers and pseudo-inverse) against one kernel per step: the
    same cycle up to the order of partial sums."""
    import torch
    ch = make()
    h0 = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, fuse_last_level=0, **kw))
    h1 = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, fuse_last_level=1, **kw))
    assert h1.info()["n"][-2] <= 1024  # the fused path applies
    mixed = kw.get("precision") == "mixed"
    dt = torch.float32 if mixed else torch.float64
    b = torch.from_numpy(np.random.default_rng(11).standard_normal(ch.n)).cuda().to(dt)
    y0, y1 = h0.vcycle(b).double().cpu().numpy(), h1.vcycle(b).double().cpu().numpy()
    assert rel_l1(y1, y0) < (1e-5 if mixed else 1e-12), rel_l1(y1, y0)
    x0, i0 = h0.gmres(restart=20, tol=1e-12, maxit=600)
    x1, i1 = h1.gmres(restart=20, tol=1e-12, maxit=600)
    torch.cuda.synchronize()
    assert i0.converged and i1.converged
    assert abs(i1.iterations - i0.iterations) <= 1, (i0.iterations, i1.iterations)
    assert rel_l1(x1.cpu().numpy(), x0.cpu().numpy()) < 1e-10
    if not mixed:
        xo, _ = oracle.Hierarchy(ch, oracle.options_for(ch, **kw)).gmres(m=20, tol=1e-12,
                                                                          maxit=600)
        assert rel_l1(x1.cpu().numpy(), xo) < 1e-10
    h0.close()
    h1.close()


def test_graph_replay_equals_direct_launches():
    """GMRES with the V-cycle replayed from a captured HIP graph (use_graph=1)
    against launching its kernels one by one (the default): the same kernels
    in the same order, so x and the iteration count are identical."""
    import torch
    ch = chaingen.delaunay_walk(20000, 5)
    kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
    out = []
    for g in (0, 1):
        h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, use_graph=g, **kw))
        x, info = h.gmres(restart=20, tol=1e-12, maxit=600)
        torch.cuda.synchronize()
        assert info.converged
        out.append((x.cpu().numpy(), info.iterations))
        h.close()
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


@pytest.mark.parametrize("name", ["delaunay20000", "tandem65"])
def test_results_bitwise_independent_of_lanes_per_row(name):
    """The V-cycle sweeps and residuals sum every row in one fixed order
    whatever the number of lanes sharing it and whatever workgroup it falls
    in, so the lanes and workgroup sizes an autotuner picks (timing-dependent,
    per process) never change a bit: one V-cycle and a whole GMRES solve are
    bitwise equal for 1, 2 and 4 lanes and 64 to 1024 threads on every
    level."""
    import torch
    if name == "delaunay20000":
        ch = chaingen.delaunay_walk(20000, 3)
        kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
    else:
        ch = chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31)
        kw = dict(r=8, max_interp=4, coarse_max=30, nu_setup=5)
    h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, autotune=0, fuse_last_level=0, **kw))
    b = torch.from_numpy(np.random.default_rng(3).standard_normal(ch.n)).cuda()
    ref_v, ref_x = None, None
    # lanes per row, then workgroup sizes (the tuner's two choices)
    for lanes, threads in ((1, 256), (2, 256), (4, 256), (4, 64), (1, 1024), (2, 512)):
        for l in range(h.levels - 1):
            h.set_lanes(l, lanes)
            h.set_threads(l, threads)
            assert h.threads(l) == threads
        v = h.vcycle(b).cpu().numpy()
        x, info = h.gmres(restart=20, tol=1e-12, maxit=300)
        x = x.cpu().numpy()
        assert info.converged
        if ref_v is None:
            ref_v, ref_x, ref_it = v, x, info.iterations
        else:
            assert np.array_equal(v, ref_v), lanes
            assert np.array_equal(x, ref_x), lanes
            assert info.iterations == ref_it


FLEX = [
    ("tandem65", lambda: chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31),
     dict(r=8, max_interp=4, coarse_max=300, nu_setup=8)),
    ("delaunay20000", lambda: chaingen.delaunay_walk(20000, 12),
     dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)),
]


@pytest.mark.parametrize("name,make,kw", FLEX, ids=[c[0] for c in FLEX])
def test_flexible_gmres(name, make, kw):
    """Flexible GMRES (right preconditioning, z_j = C v_j kept): FP64 and
    mixed reach the oracle's stationary vector, and with the FP32 V-cycles of
    the mixed form it needs no more iterations than plain FP64 GMRES plus one,
    where the left-preconditioned mixed solve needs more (the cycles'
    rounding enters the Krylov operator there: 22 against 7 iterations on
    the 65^2 tandem)."""
    import torch
    ch = make()
    xo, _ = oracle.Hierarchy(ch, oracle.options_for(ch, **kw)).gmres(m=20, tol=1e-14, maxit=600)
    its = {}
    for prec in ("fp64", "mixed"):
        for flex in (0, 1):
            h = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, precision=prec, flexible=flex,
                                                                **kw))
            _, info = h.gmres(restart=20, tol=1e-10, maxit=600)
            assert info.converged, (prec, flex)
            its[prec, flex] = info.iterations
            if flex:
                x, info = h.gmres(restart=20, tol=1e-13, maxit=600)
                torch.cuda.synchronize()
                assert info.converged
                assert rel_l1(x.cpu().numpy(), xo) < 1e-10, (prec, rel_l1(x.cpu().numpy(), xo))
            h.close()
    assert its["mixed", 1] <= its["fp64", 0] + 1, its
    assert its["mixed", 1] <= its["mixed", 0], its


RANDOM_RATES = [
    # rates of seed 14024003 (0.302, 0.230, 0.468): the drift that stops the
    # Jacobi-smoothed hierarchies from 513^2 up; with Kaczmarz sweeps 257^2
    # and 513^2 still converge (the oracle: 34 iterations to 1e-13 and 336
    # to 1e-10)
    ("tandem257_random", 257, 1e-13),
    ("tandem513_random", 513, 1e-10),
]


@pytest.mark.parametrize("name,size,tol", RANDOM_RATES, ids=[c[0] for c in RANDOM_RATES])
def test_random_rate_tandem_kaczmarz_converges(name, size, tol):
    """The largest random-rate tandems that converge: GMRES reaches tol with
    the true residual checked on the host and x is a probability vector; at
    257^2 (an oracle solve of a few seconds) x and the iteration count agree
    with the oracle's. The stationary vector is ill-conditioned here (x at
    1e-10 and at 1e-13 differ by 5e-8 in relative l1), so the comparison is
    made at 1e-13."""
    import torch
    ch = chaingen.tandem(size, *chaingen.tandem_random_rates(14024003))
    kw = dict(r=8, max_interp=4, coarse_max=300, nu_setup=8, seed=14024003,
              smoother="kaczmarz")
    hg = bamg.Hierarchy.from_chain(ch, bamg.options_for(ch, **kw))
    xg, ig = hg.gmres(restart=20, tol=tol, maxit=1000)
    torch.cuda.synchronize()
    print(f"{name}: {ig.iterations} iterations, rel residual {ig.rel_residual:.2e}", flush=True)
    assert ig.converged
    x = xg.cpu().numpy()
    A = ch.to_scipy()
    assert np.linalg.norm(x - A @ x) / np.linalg.norm(x) < 2 * tol
    assert abs(x.sum() - 1.0) < 1e-12 and x.min() > -1e-9 * x.max()
    if size <= 257:
        ho = oracle.Hierarchy(ch, oracle.options_for(ch, **kw))
        xo, io = ho.gmres(m=20, tol=tol, maxit=1000)
        assert io.converged and abs(ig.iterations - io.iterations) <= 20
        assert rel_l1(x, xo) < 1e-9
