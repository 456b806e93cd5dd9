"""Benchmark: time for BAMG-preconditioned GMRES to reach ||Bx||/||x|| < 1e-10.

One step = the whole hot path on one synthetic chain whose transition matrix
is already resident in HBM: bamg_setup (validation, hierarchy structure, one
bootstrap cycle, coarsest pseudo-inverse) followed by bamg_gmres_solve to the
tolerance. Default workload: random walk on the Delaunay triangulation of
262,144 uniform points (p_ij = 1/deg(j)), r = 8 test vectors, c = 3, 5 + 5
Jacobi sweeps, coarsening until fewer than 100 states remain (Section 7:
planar-graph level counts are to a coarsest level of < 100 variables),
GMRES(20), FP64.

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
    "delaunay262144": ("delaunay", 262144, dict(r=8, max_interp=3, nu_pre=5, nu_post=5,
                                                 nu_setup=5, coarse_max=99, seed=14024002)),
    # Table 3's rates (lam = 11/31, mu1 = mu2 = 10/31) on a 1025 x 1025 grid,
    # 7 levels down to 17 x 17 as in Section 7; 8 test-vector sweeps
    "tandem1025": ("tandem", 1025, dict(r=8, max_interp=4, coarse_max=300, nu_setup=8,
                                        seed=14024003)),
    # rates drawn U[0.2, 0.5] and normalised (seed 14024003: 0.302, 0.230, 0.468)
    "tandem1025_random": ("tandem_random", 1025, dict(r=8, max_interp=4, coarse_max=300,
                                                      nu_setup=8, seed=14024003)),
    "tandem33": ("tandem", 33, dict(r=6, max_interp=4, max_levels=3, coarse_max=1,
                                    seed=14024001)),
}


# Sources of the dominant kernel (the finest-level Jacobi sweep). The HBM
# traffic measured by hardware counters is kept in profiles/ together with
# the digest of these files; after any change to them it no longer applies.
KERNEL_SOURCES = ("paper_1402_4005_amd/csrc/k_sparse.hip",
                  "paper_1402_4005_amd/csrc/device_common.h")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none for this
    workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"k_jacobi_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json: "):
                d = json.loads(line[len("traffic-json: "):])
                if d.get("source_digest") == kernel_digest() and d.get("precision") == precision:
                    return d
    return None


def make_chain(kind, size, seed):
    import chaingen
    if kind == "delaunay":
        return chaingen.delaunay_walk(size, seed)
    if kind == "tandem_random":
        return chaingen.tandem(size, *chaingen.tandem_random_rates(seed))
    return chaingen.tandem(size, 11 / 31, 10 / 31, 10 / 31)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="delaunay262144", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--setup-cycles", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--vcycle-reps", type=int, default=100)
    ap.add_argument("--maxit", type=int, default=1000)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision comparison run")
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

    kind, size, wopts = WORKLOADS[args.workload]
    ch = make_chain(kind, size, wopts["seed"])
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(ch.indptr).to(dev)
    ci = torch.from_numpy(ch.indices).to(dev)
    va = torch.from_numpy(ch.data).to(dev)
    stream = torch.cuda.current_stream()

    def options(precision):
        return bamg.options_for(ch, precision=precision, setup_cycles=args.setup_cycles,
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

    # kernel timing: the same K steps again with HIP events around every run of
    # finest-level Jacobi sweeps (event recording bypasses the V-cycle graph)
    launches = 0
    kms = 0.0
    kbytes = 0.0
    for _ in range(args.steps):
        hp, _, _, prof = step(opts, profile=True)
        launches += prof[0]
        kms += prof[1]
        kbytes += prof[2]
        hp.close()

    # untimed: accuracy and split of the last step, V-cycle bandwidth
    hinfo = last.info()
    xs = x.cpu().numpy()
    extra = {}
    if kind == "delaunay":
        deg = ch.extra["deg"]
        pi = deg / deg.sum()
        extra["x_err_rel_l1_vs_closed_form"] = float(np.abs(xs - pi).sum())
    torch.cuda.synchronize()
    ts = time.perf_counter()
    hs = bamg.Hierarchy(rp, ci, va, ch.geom, opts, stream=stream)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - ts) * 1e3
    hs.close()
    vcycle = vcycle_rate(opts)

    # the mixed-precision form on the same workload: FP32 setup and V-cycles,
    # FP64 Krylov, residual, normalisation and coarsest solve
    mixed = None
    if args.precision == "fp64" and not args.no_mixed:
        mopts = options("mixed")
        mms, mh, mx, minfos = timed(mopts)
        mxs = mx.cpu().numpy()
        mixed = {
            "ms_per_step": round(mms, 3),
            "speedup_vs_fp64": round(ms_per_step / mms, 3),
            "iterations": [i.iterations for i in minfos],
            "converged": [bool(i.converged) for i in minfos],
            "x_rel_l1_vs_fp64": float(np.abs(mxs - xs).sum() / np.abs(xs).sum()),
            "vcycle": vcycle_rate(mopts),
        }
        mh.close()
    last.close()

    traffic = measured_traffic(args.workload, args.precision)
    achieved = (kbytes / launches) / (kms / launches * 1e-3) / 1e9 if launches else None
    roofline = {
        "kernel": "k_jacobi (finest-level weighted-Jacobi sweep, CSR, 8 lanes/row)",
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "traffic_vs_algorithmic": (round(traffic["bytes_per_launch"] / (kbytes / launches), 3)
                                   if traffic and launches else None),
        "launches": launches,
        "avg_us": round(kms / launches * 1e3, 3) if launches else None,
        "bytes_per_launch": kbytes / launches if launches else None,
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ko = oracle.options_for(ch, setup_cycles=args.setup_cycles,
                                **{k: v for k, v in wopts.items()})
        tc = time.perf_counter()
        ho = oracle.Hierarchy(ch, ko)
        xo, io = ho.gmres(m=args.restart, tol=args.tol, maxit=1000)
        cpu_ms = (time.perf_counter() - tc) * 1e3
        cpu = {"value": round(cpu_ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"one full solve of the same workload (setup + GMRES to {args.tol:g}), "
                         f"single thread, {io.iterations} iterations",
               "x_rel_l1_gpu_vs_oracle": float(np.abs(xs - xo).sum() / np.abs(xo).sum())}

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
        },
        "iterations": it,
        "converged": [bool(i.converged) for i in infos],
        "setup_ms": round(setup_ms, 3),
        "vcycle": vcycle,
        "mixed": mixed,
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
