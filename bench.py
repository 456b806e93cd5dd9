"""Benchmark: time for BAMG-preconditioned GMRES to reach ||Bx||/||x|| < 1e-10.

One step = the whole hot path on one synthetic chain whose transition matrix
is already resident in HBM: bamg_setup (validation, hierarchy structure, one
bootstrap cycle, coarsest pseudo-inverse) followed by bamg_gmres_solve to the
tolerance. Default workload: the tandem queueing network of Section 7
(Table 3's rates lam = 11/31, mu1 = mu2 = 10/31) on a 2049 x 2049 grid
(4,198,401 states, the largest single-GPU size), r = 8 test vectors, c = 4,
3 + 3 Jacobi sweeps, 8 setup sweeps, geometric coarsening down to 33 x 33
(7 levels), GMRES(20), FP64; beside it the same steps in mixed precision and
with the learned interpolation weights. Its finest operator and vectors
(about 0.5 GB) exceed the 256 MB Infinity Cache, so the sweep's bandwidth is
HBM bandwidth. The random-rate tandems of the same sizes (rates drawn
U[0.2, 0.5] and normalised) are run too, untimed and capped at 100
iterations, and reported with their convergence status.

Prints one JSON line. `value` is the time to tolerance in ms (lower is
better), over K timed steps. `roofline` covers the dominant kernel (the
finest-level weighted Jacobi sweep of the V-cycle), timed with HIP events on
its launch stream over a second pass of the same K steps; `cpu_baseline` is
the FP64 CPU oracle on the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X published HBM3E bandwidth
METRIC = ("time to \u2016Bx\u2016/\u2016x\u2016<1e-10 + V-cycle HBM GB/s; "
          "mixed/learned vs plain FP64")

WORKLOADS = {
    # name: (kind, size, options)
    # Table 3's rates on a 2049 x 2049 grid; coarsening stops at 33 x 33 (7
    # levels): with a 17 x 17 coarsest level the two deepest Galerkin levels
    # lose the sign structure Jacobi needs and GMRES stalls at this size
    # validate = 3: the chain is still checked for stochasticity and strong
    # connectivity inside the timed step, but the search (latency-bound over
    # the grid's ~4000-hop diameter) is joined at the end of the solve rather
    # than the setup, so it overlaps both
    "tandem2049": ("tandem", 2049, dict(r=8, max_interp=4, coarse_max=1100, nu_setup=8,
                                        seed=14024101, validate=3)),
    "delaunay262144": ("delaunay", 262144, dict(r=8, max_interp=3, nu_pre=5, nu_post=5,
                                                 nu_setup=5, coarse_max=99, seed=14024002,
                                                 validate=3)),
    # Table 3's rates on a 1025 x 1025 grid, 7 levels down to 17 x 17 as in
    # Section 7; 8 test-vector sweeps
    "tandem1025": ("tandem", 1025, dict(r=8, max_interp=4, coarse_max=300, nu_setup=8,
                                        seed=14024003)),
    # rates drawn U[0.2, 0.5] and normalised (seed 14024003: 0.302, 0.230, 0.468)
    "tandem1025_random": ("tandem_random", 1025, dict(r=8, max_interp=4, coarse_max=300,
                                                      nu_setup=8, seed=14024003)),
    "tandem2049_random": ("tandem_random", 2049, dict(r=8, max_interp=4, coarse_max=1100,
                                                      nu_setup=8, seed=14024101)),
    "tandem33": ("tandem", 33, dict(r=6, max_interp=4, max_levels=3, coarse_max=1,
                                    seed=14024001)),
}

# untimed convergence status of the random-rate tandems (rates from each seed)
STATUS_RUNS = [("tandem1025_random", 1025, 14024003)] + \
    [("tandem2049_random", 2049, s) for s in range(14024101, 14024106)]


# Sources of the two profiled kernels: the finest-level Jacobi sweep of the
# V-cycle and the round kernel of the coarsest-level Jacobi SVD. The HBM
# traffic measured by hardware counters is kept in profiles/ together with
# the digest of these files; after any change to them it no longer applies.
KERNEL_SOURCES = {
    "k_jacobi": ("paper_1402_4005_amd/csrc/k_sparse.hip", "paper_1402_4005_amd/csrc/sparse_row.h",
                 "paper_1402_4005_amd/csrc/device_common.h"),
    "k_block_jacobi_round": ("paper_1402_4005_amd/csrc/k_dense.hip",
                             "paper_1402_4005_amd/csrc/device_common.h"),
}


def progress(msg):
    """One line on stderr when a phase of the run ends (the JSON result is
    the only line on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_digest(kernel="k_jacobi"):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, kernel="k_jacobi"):
    """HBM bytes per launch of a profiled kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none for this
    workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json: "):
                d = json.loads(line[len("traffic-json: "):])
                if (d.get("source_digest") == kernel_digest(kernel)
                        and d.get("precision") == precision):
                    return d
    return None


def make_chain(kind, size, seed):
    import chaingen
    if kind == "delaunay":
        return chaingen.delaunay_walk(size, seed)
    if kind == "tandem_random":
        return chaingen.tandem(size, *chaingen.tandem_random_rates(seed))
    return chaingen.tandem(size, 11 / 31, 10 / 31, 10 / 31)


# training chains of the learned form, per family: (kind, size, seed)
LEARN_TRAIN = {
    "delaunay": [("delaunay", n, 100 + i) for i, n in enumerate([4096, 8192, 16384, 32768,
                                                                  65536])],
    "tandem": [("tandem", n, 0) for n in (33, 65, 129, 257)],
}


def batch_members(count, master_seed):
    """The batched workload: chain k uses numpy's generator seeded with
    (master_seed, k). Even k: tandem queue on an N x N grid, N uniform in
    17..257, rates uniform in [0.2, 0.5] normalised; odd k: Delaunay random
    walk on 2^U[10, 16] uniform points. Options per family as in Section 7
    (tandem: r = 8, c = 4, 3 + 3 sweeps, 7+ levels to 17 x 17; planar: c = 3,
    5 + 5 sweeps, coarsest < 100), FP32 cycles with FP64 Krylov."""
    import numpy as np
    import chaingen
    out = []
    for k in range(count):
        rng = np.random.default_rng([master_seed, k])
        if k % 2 == 0:
            N = int(rng.integers(17, 258))
            r = rng.uniform(0.2, 0.5, 3)
            r = r / r.sum()
            ch = chaingen.tandem(N, *r)
            kw = dict(r=8, max_interp=4, coarse_max=300 if N >= 65 else 99, nu_setup=8)
        else:
            n = int(round(2 ** rng.uniform(10, 16)))
            ch = chaingen.delaunay_walk(n, int(rng.integers(1 << 31)))
            kw = dict(r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5, coarse_max=99)
        out.append((ch, kw))
    return out


def run_batch(args):
    """Many chains per step: bamg_setup_batched + bamg_gmres_solve_batched."""
    import numpy as np
    import torch
    import paper_1402_4005_amd as bamg
    tg = time.perf_counter()
    mem = batch_members(args.batch, 14024004)
    gen_s = time.perf_counter() - tg
    chains = [c for c, _ in mem]
    opts = [bamg.options_for(c, precision=args.precision if args.precision != "fp64" else "mixed",
                             **kw) for c, kw in mem]

    arrays = bamg.Batch.upload(chains)  # inputs resident before the timed region
    split = [0.0, 0.0]  # setup, solve (ms, summed over the timed steps)

    def step():
        ta = time.perf_counter()
        b = bamg.Batch(chains, opts, nstreams=args.streams, arrays=arrays)
        b.set_solver(args.batch_solver)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        xs, infos, sts = b.gmres(restart=args.restart, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        split[0] += (tb - ta) * 1e3
        split[1] += (time.perf_counter() - tb) * 1e3
        return b, infos, sts

    for _ in range(args.warmup):
        step()[0].close()
    torch.cuda.synchronize()
    split[:] = [0.0, 0.0]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b, infos, sts = step()
        b.close()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    nconv = sum(1 for s in sts if s == 0)
    states = sum(c.n for c in chains)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        tc = time.perf_counter()
        done, done_nnz = 0, 0
        for c, kw in mem:
            if time.perf_counter() - tc > 15.0:
                break
            try:
                ho = oracle.Hierarchy(c, oracle.options_for(c, **kw))
                ho.gmres(m=args.restart, tol=args.tol, maxit=args.maxit)
            except Exception:
                pass
            done += 1
            done_nnz += c.nnz
        el = time.perf_counter() - tc
        tot_nnz = sum(c.nnz for c in chains)
        cpu = {"value": round(el * 1e3 * tot_nnz / max(done_nnz, 1), 1), "unit": "ms",
               "cores": 1, "kind": "oracle",
               "sample": f"oracle setup+GMRES of the first {done} chains ({done_nnz} nnz of "
                         f"{tot_nnz}) in {el:.1f} s, scaled by nonzeros to the whole batch"}
    line = {
        "metric": METRIC, "value": round(ms, 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"batch{args.batch}", "chains": args.batch, "states": states,
                   "nnz_A": sum(c.nnz for c in chains), "streams": args.streams or 4,
                   "solver": args.batch_solver,
                   "tol": args.tol, "restart": args.restart},
        "chains_per_s": round(args.batch / (ms * 1e-3), 1),
        "setup_ms": round(split[0] / args.steps, 1), "solve_ms": round(split[1] / args.steps, 1),
        "converged": nconv,
        "failed": {str(s): sum(1 for x in sts if x == s) for s in set(sts) if s != 0},
        "iterations_median": float(np.median([i.iterations for i, s in zip(infos, sts) if s == 0]))
        if nconv else None,
        "host_generation_s": round(gen_s, 1),
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def cpu_baseline(args, kind, size, wopts, ch, xs):
    """The FP64 oracle's time for the whole method (setup + GMRES to tol), on
    the host cores, single thread and with every thread of the process's
    share (OpenMP over independent row loops: same results). On the 2049^2
    tandem the serial oracle needs minutes (its 1089-state coarsest dense SVD
    alone over one), so the sample is the same chain family and options at
    1025^2 with a 17^2 coarsest level, scaled by nonzeros."""
    import numpy as np
    import oracle
    nthr = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if kind == "tandem" and size > 1025:
        sch = make_chain(kind, 1025, wopts["seed"])
        skw = dict(wopts, coarse_max=300)
        scale = ch.nnz / sch.nnz
        what = (f"oracle setup + GMRES to {args.tol:g} on the 1025^2 tandem (Table 3 rates, "
                f"17^2 coarsest level), scaled by nonzeros x{scale:.2f} to the {size}^2 chain")
    else:
        sch, skw, scale = ch, dict(wopts), 1.0
        what = f"one full solve of the same workload (setup + GMRES to {args.tol:g})"
    skw.pop("validate", None)  # the oracle validates in its own setup
    ko = oracle.options_for(sch, setup_cycles=args.setup_cycles, **skw)
    times, its, xo = [], None, None
    for threads in (1, nthr):
        oracle.set_threads(threads)
        tc = time.perf_counter()
        ho = oracle.Hierarchy(sch, ko)
        xo, io = ho.gmres(m=args.restart, tol=args.tol, maxit=1000)
        times.append((time.perf_counter() - tc) * 1e3 * scale)
        its = io.iterations
        del ho
    out = {"value": round(times[0], 1), "unit": "ms", "cores": 1, "kind": "oracle",
           "sample": f"{what}, {its} iterations; value is the single-thread time",
           "value_all_threads": round(times[1], 1), "threads": nthr}
    if sch is ch:
        out["x_rel_l1_gpu_vs_oracle"] = float(np.abs(xs - xo).sum() / np.abs(xo).sum())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tandem2049", choices=sorted(WORKLOADS) + ["batch"])
    ap.add_argument("--coarsening", default=None, choices=["mis", "cr"],
                    help="algebraic C/F splitting of a workload without geometry "
                         "(default: the workload's own)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--setup-cycles", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--vcycle-reps", type=int, default=100)
    ap.add_argument("--maxit", type=int, default=1000)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision comparison run")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-interpolation comparison run")
    ap.add_argument("--no-status", action="store_true",
                    help="skip the convergence status of the random-rate tandems")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1 = time the lanes per CSR row of every level's sweeps at setup")
    ap.add_argument("--graph", action="store_true",
                    help="replay the V-cycle inside GMRES from a captured HIP graph instead "
                         "of launching its kernels one by one")
    ap.add_argument("--batch", type=int, default=512,
                    help="chains of the batched workload (--workload batch)")
    ap.add_argument("--streams", type=int, default=0, help="library streams of a batch")
    ap.add_argument("--batch-solver", default="auto", choices=["auto", "persistent", "streams"],
                    help="batched solve: small chains in one persistent launch and the others "
                         "per chain on the streams (auto), all in the launch, or all on streams")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB (the known "
                         "byte count that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the method is benchmarked on one MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        nel = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nel * 8, "bytes_written": nel * 8,
                          "copies": 5}))
        return

    import paper_1402_4005_amd as bamg

    if args.workload == "batch":
        run_batch(args)
        return
    kind, size, wopts = WORKLOADS[args.workload]
    if args.coarsening:
        wopts = dict(wopts, coarsening=args.coarsening)
    ch = make_chain(kind, size, wopts["seed"])
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(ch.indptr).to(dev)
    ci = torch.from_numpy(ch.indices).to(dev)
    va = torch.from_numpy(ch.data).to(dev)
    stream = torch.cuda.current_stream()

    def options(precision):
        return bamg.options_for(ch, precision=precision, setup_cycles=args.setup_cycles,
                                autotune=args.autotune, use_graph=1 if args.graph else 0,
                                **wopts)

    def step(opts, profile=False):
        h = bamg.Hierarchy(rp, ci, va, ch.geom, opts, stream=stream)
        if profile:
            h.profile_begin(0)
        x, info = h.gmres(restart=args.restart, tol=args.tol, maxit=args.maxit, stream=stream)
        prof = h.profile_end() if profile else None
        return h, x, info, prof

    def timed(opts):
        for _ in range(args.warmup):
            h, x, info, _ = step(opts)
            h.close()
        # timed region: K whole steps, device-synchronised on both sides
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            h, x, info, _ = step(opts)
            infos.append(info)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) * 1e3 / args.steps, h, x, infos

    def vcycle_rate(opts):
        hs = bamg.Hierarchy(rp, ci, va, ch.geom, opts, stream=stream)
        dt = torch.float64 if opts.precision == 0 else torch.float32
        b = torch.randn(ch.n, dtype=torch.float64, device=dev).to(dt)
        xv = torch.empty_like(b)
        hs.vcycle(b, xv)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.vcycle_reps):
            hs.vcycle(b, xv)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.vcycle_reps
        nbytes = hs.vcycle_bytes()
        hs.close()
        return {"ms": round(ms, 4), "bytes": nbytes, "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}

    opts = options(args.precision)
    progress(f"{args.workload}: {ch.n} states built, {args.warmup} warm-up + {args.steps} timed steps")
    try:
        ms_per_step, last, x, infos = timed(opts)
    except bamg.BamgError as e:
        # the method itself failed on this chain (setup or solve status < 0)
        print(json.dumps({"metric": METRIC, "value": None, "unit": "ms", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup,
                          "higher_is_better": False, "dtype": args.precision,
                          "data": "synthetic", "config": {"workload": args.workload,
                                                          "n": ch.n},
                          "error": {"status": e.code, "message": str(e)}}))
        return

    progress(f"timed steps done: {ms_per_step:.3f} ms per step")
    # kernel timing: the same K steps again with HIP events around every run of
    # finest-level Jacobi sweeps (event recording bypasses the V-cycle graph),
    # and K setups with events around the coarsest Jacobi SVD's round launches
    launches = 0
    kms = 0.0
    kbytes = 0.0
    for _ in range(args.steps):
        hp, _, _, prof = step(opts, profile=True)
        launches += prof[0]
        kms += prof[1]
        kbytes += prof[2]
        hp.close()
    svd = [0, 0.0, 0.0]
    popts = options(args.precision)
    popts.profile_setup = 1
    for _ in range(args.steps):
        hq = bamg.Hierarchy(rp, ci, va, ch.geom, popts, stream=stream)
        for i, v in enumerate(hq.profile_end()):
            svd[i] += v
        hq.close()

    # untimed: accuracy and split of the last step, V-cycle bandwidth
    hinfo = last.info()
    hinfo_lanes = last.lanes(0)
    hinfo_threads = last.threads(0)
    xs = x.cpu().numpy()
    extra = {}
    if kind == "delaunay":
        deg = ch.extra["deg"]
        pi = deg / deg.sum()
        extra["x_err_rel_l1_vs_closed_form"] = float(np.abs(xs - pi).sum())
    # the setup's own time inside the timed steps (bamg_setup entry to
    # return; with validation joined by the solve, the search is not in it)
    setup_ms = float(np.mean([i.t_setup_ms for i in infos]))
    vcycle = vcycle_rate(opts)
    progress(f"kernel timing and V-cycle rate done ({vcycle['ms']} ms per V-cycle)")

    # the learned form: a network trained (untimed) on BAMG^2 corrections of
    # smaller chains of the same family, then one-cycle setups with it
    learned_line = None
    if args.precision == "fp64" and not args.no_learned and kind in LEARN_TRAIN:
        from paper_1402_4005_amd import learned as lmod
        tl = time.perf_counter()
        tchains = [make_chain(k2, s2, sd2) for k2, s2, sd2 in LEARN_TRAIN[kind]]
        hkw = {k: v for k, v in wopts.items() if k != "seed"}
        hkw["coarse_max"] = min(hkw.get("coarse_max", 300), 300)
        LX, LT, LM = lmod.harvest(tchains, **hkw)
        net, losses = lmod.train(LX, LT, LM, epochs=120)
        train_s = time.perf_counter() - tl
        lopts = options(args.precision)
        lopts.learned = bamg.LEARNED_USE
        lopts.mlp = net.h.value
        # iteration fallback: past plain BAMG's count plus two, the hierarchy
        # is rebuilt with the exact fits and GMRES continues
        lopts.learned_max_iters = max(i.iterations for i in infos) + 2
        lms, lh, lx, linfos = timed(lopts)
        lxs = lx.cpu().numpy()
        nm, nl = lh.learned_stats()
        learned_line = {
            "ms_per_step": round(lms, 3),
            "speedup_vs_fp64": round(ms_per_step / lms, 3),
            "iterations": [i.iterations for i in linfos],
            "converged": [bool(i.converged) for i in linfos],
            "x_rel_l1_vs_fp64": float(np.abs(lxs - xs).sum() / np.abs(xs).sum()),
            "mlp_rows": nm, "ls_fallback_rows": nl,
            "iteration_fallbacks": sum(i.mlp_fallback for i in linfos),
            "fallback_after_iterations": lopts.learned_max_iters,
            "training": {"chains": [f"{k2}{s2}" for k2, s2, _ in LEARN_TRAIN[kind]],
                         "samples": int(LX.shape[0]), "epochs": 240,
                         "loss_first_last": [round(float(losses[0]), 5),
                                             round(float(losses[-1]), 5)],
                         "seconds": round(train_s, 1)},
        }
        lh.close()
        net.close()
        progress(f"learned form done: {lms:.3f} ms per step")

    # BAMG^2 (two setup cycles, Section 7), whose second cycle the learned
    # weights stand in for
    bamg2 = None
    if args.precision == "fp64" and not args.no_learned:
        b2opts = options(args.precision)
        b2opts.setup_cycles = 2
        b2ms, b2h, _, b2infos = timed(b2opts)
        b2h.close()
        bamg2 = {"ms_per_step": round(b2ms, 3), "speedup_vs_fp64": round(ms_per_step / b2ms, 3),
                 "iterations": [i.iterations for i in b2infos],
                 "converged": [bool(i.converged) for i in b2infos]}
        if learned_line:
            learned_line["speedup_vs_bamg2"] = round(b2ms / learned_line["ms_per_step"], 3)
        progress(f"BAMG^2 done: {b2ms:.3f} ms per step")

    # the mixed-precision form on the same workload: FP32 setup and V-cycles,
    # FP64 Krylov, residual, normalisation and coarsest solve; flexible GMRES,
    # so the FP32 cycles' rounding does not enter the minimised residual
    mixed = None
    if args.precision == "fp64" and not args.no_mixed:
        mopts = options("mixed")
        mopts.flexible = 1
        mms, mh, mx, minfos = timed(mopts)
        mxs = mx.cpu().numpy()
        mixed = {
            "ms_per_step": round(mms, 3),
            "speedup_vs_fp64": round(ms_per_step / mms, 3),
            "iterations": [i.iterations for i in minfos],
            "converged": [bool(i.converged) for i in minfos],
            "x_rel_l1_vs_fp64": float(np.abs(mxs - xs).sum() / np.abs(xs).sum()),
            "krylov": "flexible GMRES (right preconditioning)",
            "vcycle": vcycle_rate(mopts),
        }
        mh.close()
        progress(f"mixed precision done: {mms:.3f} ms per step")
    last.close()

    # random-rate tandems (configurations whose rates are drawn): setup and
    # at most 100 GMRES iterations each, untimed, with the outcome
    status = None
    if args.workload == "tandem2049" and not args.no_status:
        import chaingen
        status = []
        for name, N, sd in STATUS_RUNS:
            rates = chaingen.tandem_random_rates(sd)
            sch = chaingen.tandem(N, *rates)
            sopts = bamg.options_for(sch, **dict(WORKLOADS[name][2], seed=sd))
            entry = {"workload": name, "rate_seed": sd,
                     "rates": [round(float(r), 4) for r in rates]}
            try:
                hst = bamg.Hierarchy.from_chain(sch, sopts, on_device=True, stream=stream)
                _, sinfo = hst.gmres(restart=args.restart, tol=args.tol, maxit=100, stream=stream)
                entry.update(converged=bool(sinfo.converged), iterations=sinfo.iterations,
                             rel_residual=float(f"{sinfo.rel_residual:.3g}"))
                hst.close()
            except bamg.BamgError as e:
                entry["error"] = str(e)
            status.append(entry)
            progress(f"status of {name} (rate seed {sd}) done")

    def roofline_of(name, kernel, n_launch, ms_tot, bytes_tot):
        if not n_launch:
            return None
        traffic = measured_traffic(args.workload, args.precision, kernel)
        achieved = (bytes_tot / n_launch) / (ms_tot / n_launch * 1e-3) / 1e9
        return {
            "kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic["bytes_per_launch"] if traffic else None,
            "traffic_vs_algorithmic": (round(traffic["bytes_per_launch"] / (bytes_tot / n_launch),
                                             3) if traffic else None),
            "launches": n_launch, "avg_us": round(ms_tot / n_launch * 1e3, 3),
            "bytes_per_launch": bytes_tot / n_launch,
            "ms_per_step": round(ms_tot / args.steps, 3),
        }

    sweep_roof = roofline_of(f"k_jacobi (finest-level weighted-Jacobi sweep, CSR, {hinfo_lanes} "
                             f"lanes/row, {hinfo_threads} threads/workgroup)", "k_jacobi",
                             launches, kms, kbytes)
    svd_roof = roofline_of("k_block_jacobi_round (coarsest-level block Jacobi SVD, one launch "
                           "per round)", "k_block_jacobi_round", int(svd[0]), svd[1], svd[2])
    # the roofline object covers whichever of the two takes more time per step
    roofline = sweep_roof
    if svd_roof and (not sweep_roof or svd_roof["ms_per_step"] > sweep_roof["ms_per_step"]):
        roofline = svd_roof

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, kind, size, wopts, ch, xs)
        progress("oracle baseline done")

    it = [i.iterations for i in infos]
    line = {
        "metric": METRIC,
        "value": round(ms_per_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n": ch.n, "nnz_A": ch.nnz, "levels": hinfo["levels"], "n_l": hinfo["n"],
            "oc": round(hinfo["oc"], 3), "og": round(hinfo["og"], 3),
            "r": opts.r, "c": opts.max_interp, "sweeps": f"{opts.nu_pre}+{opts.nu_post}",
            "setup_cycles": opts.setup_cycles, "restart": args.restart, "tol": args.tol,
            "precision": args.precision,
            "coarsening": {0: "geometric", 1: "mis", 2: "cr"}[opts.coarsening],
            "validation": {0: "none", 1: "joined by the setup", 2: "joined by the setup",
                           3: "joined by the solve"}[opts.validate],
            "autotune": ("lanes per row and workgroup size of each level's sweeps, timed "
                         "during the warm-up steps and reused by the timed steps (the "
                         "choices change speed only, not results)") if args.autotune else "off",
        },
        "iterations": it,
        "converged": [bool(i.converged) for i in infos],
        "setup_ms": round(setup_ms, 3),
        "vcycle": vcycle,
        "mixed": mixed,
        "learned": learned_line,
        "bamg2": bamg2,
        "roofline": roofline,
        "roofline_finest_sweep": sweep_roof,
        "roofline_coarsest_svd": svd_roof,
        "cpu_baseline": cpu,
        "random_rate_status": status,
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
