#!/usr/bin/env python3
"""DF-J/K build throughput on one MI355X.

One step is one whole job on the 32-water cluster (960 AO, 2,784 aux, 160
occupied orbitals; 10 A box, O-O >= 2.6 A, geometry seed 1): host
preparation, Schwarz screening, three-centre integrals, metric, Cholesky,
L^{-1}, whitening, then 10 SCF-like J/K builds with perturbed occupied
orbitals.  `value` is completed builds per second over the timed steps
(setup included); the steady-state time of one build is reported beside it.
FP64 is the headline; FP32 and BF16x3 K contractions are timed the same way
and their energy errors against the FP64 path are reported.

The roofline entry is the dominant kernel (the FP64 K contraction, X X^T on
FP64 MFMA), timed live by HIP events the library records on its own stream.
The CPU baseline is the FP64 oracle timed on a bounded sample of the same
job and scaled to builds per second (see cpu_baseline.sample).

Beside the headline line the JSON carries the 128-water cluster (3,840 AO,
11,136 aux, nocc 640, Schwarz 1e-10, K streamed over aux slabs; `water128`,
skipped with --no-large) and a continuous-batching serving stream (`serving`).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NBUILDS = 10
PEAK_F64_TFLOPS = 78.6
PEAK_F32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_BYTES = 8.0e12
PEAK_INT8_TOPS = 5000.0          # dense int8 MFMA
I8_PRODUCTS = 15                 # int8 slice products per FP64-equivalent product (five slices, orders <= 4)
I8F_PRODUCTS = 10                # the same for int8_fast (orders <= 3)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "water32.json")


def golden_errors(E, K_last):
    """Errors of one mode's water32 job against the oracle's stored values
    (tests/golden/water32.json, written by the CPU oracle alone): |dE_J|,
    |dE_K| of builds 0 and 9, max |dK| over the stored K rows of build 9."""
    import numpy as np
    g = json.load(open(GOLDEN))
    dEJ = max(abs(E[int(k)][0] - b["E_J"]) for k, b in g["builds"].items())
    dEK = max(abs(E[int(k)][1] - b["E_K"]) for k, b in g["builds"].items())
    last = str(len(E) - 1)
    dK = float(np.abs(K_last[g["rows"]] - np.asarray(g["builds"][last]["K_rows"])).max()) if last in g["builds"] else None
    return {"max_abs_dE_J_vs_oracle": float(dEJ), "max_abs_dE_K_vs_oracle": float(dEK),
            "max_abs_dK_rows_vs_oracle": dK, "builds_compared": sorted(int(k) for k in g["builds"])}


def committed_traffic(shape):
    """HBM bytes per launch of the FP64 K kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernel source or its
    launch shape (tile, split count) changed since those counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_syrk_f64_water32.md")
    src = os.path.join(ROOT, "paper_2404_09452_amd", "csrc", "syrk_f64.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    b = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    k = re.search(r"kernel_shape:\s*(\d+)x(\d+)", text)
    if not b or not h or h.group(1) != sha or not k:
        return None
    if (int(k.group(1)), int(k.group(2))) != (shape["k_tile"], shape["nsplit"]):
        return None
    return int(b.group(1))


def committed_direct_flops():
    """FP64 VALU flops per direct build (per Schwarz threshold) from the
    committed rocprofv3 counter summary, or {} when the direct kernels'
    source changed since those counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "direct_jk_water32.md")
    src = os.path.join(ROOT, "paper_2404_09452_amd", "csrc", "direct.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return {}
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    if not h or h.group(1) != sha:
        return {}
    return {float(t): float(f) for t, f in re.findall(r"fp64_valu_flops_per_build\[tau=([0-9.e+-]+)\]:\s*([0-9.e+]+)", text)}


def direct_bench(mol, Cd, taus=(1e-10, 1e-12), nbuild=5, E_df=None, S=None):
    """Four-centre direct J/K (exact exchange) on the same molecule and
    orbitals: ms per build (HIP events on the stream the builds run on),
    screened quartets, and the FP64 VALU roofline fraction from committed
    counters."""
    import numpy as np
    import torch
    from paper_2404_09452_amd.dfjk import Plan
    flops = committed_direct_flops()
    out = {}
    for tau in taus:
        t0 = time.perf_counter()
        plan = Plan.from_molecule(mol, schwarz_thresh=tau).screen().direct_setup()
        torch.cuda.synchronize()
        setup_ms = 1000.0 * (time.perf_counter() - t0)
        st = plan.direct_stats()
        plan.direct_build(C=Cd[0])
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nbuild)]
        for b in range(nbuild):
            ev[2 * b].record(stream)
            J, K, E = plan.direct_build(C=Cd[b % len(Cd)], stream=stream)
            ev[2 * b + 1].record(stream)
        torch.cuda.synchronize()
        ms = [ev[2 * b].elapsed_time(ev[2 * b + 1]) for b in range(nbuild)]
        med = float(np.median(ms))
        Ed = E.cpu().numpy()
        r = {"ms_per_build_median": round(med, 3), "ms_per_build_min": round(float(np.min(ms)), 3),
             "builds_per_s": round(1000.0 / med, 3), "setup_ms": round(setup_ms, 2),
             "pairs_per_class_ss_ps_pp_ds_dp_dd": st["pairs"], "quartets": st["quartets"],
             "quartets_per_s": round(st["quartets"] / (med * 1e-3), 1),
             "E_J": float(Ed[0]), "E_K": float(Ed[1])}
        if E_df is not None:
            k = (nbuild - 1) % len(Cd)
            r["E_exact_minus_E_DF"] = [float(Ed[0] - E_df[k][0]), float(Ed[1] - E_df[k][1])]
        f = flops.get(tau)
        if f:
            ach = f / (med * 1e-3) / 1e12
            r["roofline"] = {"bound": "alu", "unit": "TFLOP/s", "peak": PEAK_F64_TFLOPS,
                             "achieved": round(ach, 3), "frac": round(ach / PEAK_F64_TFLOPS, 4),
                             "flops_per_build": f,
                             "flops_source": "profiles/direct_jk_water32.md (FP64 VALU instruction counters)"}
        if S is not None and tau == taus[0]:
            r["incremental"] = direct_delta_bench(plan, Cd[0], S, med, nbuild)
        out["tau_%g" % tau] = r
        plan.close()
        del J, K, E
    torch.cuda.empty_cache()
    return out


def direct_delta_bench(plan, C0, S, full_ms, nbuild):
    """Incremental direct builds J0, K0 + J, K(D - D0) with the
    density-weighted screen, for a step like the headline sequence's
    (eps 1e-2) and a late-iteration step (eps 1e-4); HIP events on the
    stream the builds run on."""
    import numpy as np
    import torch
    import workload as W
    C0h = C0.cpu().numpy()
    D0 = 2.0 * C0 @ C0.T
    J0, K0, _ = plan.direct_build(D=D0)
    out = {}
    stream = torch.cuda.current_stream()
    for eps in (1e-2, 1e-4):
        C1 = torch.as_tensor(W.perturbed_orbitals(C0h, S, 1, eps=eps, seed=4242), device="cuda")
        D1 = 2.0 * C1 @ C1.T
        _, _, Ef = plan.direct_build(D=D1)
        plan.direct_build_delta(D1, D0, J0, K0)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nbuild)]
        for b in range(nbuild):
            ev[2 * b].record(stream)
            _, _, E = plan.direct_build_delta(D1, D0, J0, K0, stream=stream)
            ev[2 * b + 1].record(stream)
        torch.cuda.synchronize()
        med = float(np.median([ev[2 * b].elapsed_time(ev[2 * b + 1]) for b in range(nbuild)]))
        dE = (E - Ef).abs().cpu().numpy()
        out["eps_%g" % eps] = {"ms_per_build_median": round(med, 3), "speedup_vs_full": round(full_ms / med, 2),
                               "max_abs_dD": float((D1 - D0).abs().max()),
                               "abs_dE_vs_full_build": [float(dE[0]), float(dE[1])]}
    return out


def batching_bench(nmol=16, reps=3, seed=7):
    """Batching of uneven molecules: nmol water clusters of 1..12 molecules
    (seeded sizes), set up one by one against one dfjk_setup_batch (pair
    records and three-centre integrals of all molecules in shared launches),
    then their FP64 builds one by one against one dfjk_build_batch (grouped
    K, reductions and energies) and its HIP-graph replay.  Orbitals are
    random orthonormal columns of nocc = 5 per water (only shapes matter to
    the timing); batched results are checked against the single ones.  The
    best of `reps` timings of each form; then the builds once more in
    int8_fast, one by one and batched."""
    import numpy as np
    import torch
    import workload as W
    from paper_2404_09452_amd import dfjk as G

    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.integers(1, 13, size=nmol)]
    mols = []
    for k, n in enumerate(sizes):
        z, x = W.water_cluster(n, 4.0 + 1.5 * n ** (1.0 / 3.0), 100 + k) if n > 1 else W.water_monomer()
        mols.append(W.make_molecule(z, x))
    Cs = [torch.as_tensor(np.linalg.qr(rng.standard_normal((m.nao, m.nelec // 2)))[0], device="cuda")
          for m in mols]

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0), out

    single_setup, batch_setup = [], []
    plans = None
    for _ in range(reps):
        ps = [G.Plan.from_molecule(m, schwarz_thresh=1e-14).screen() for m in mols]
        t, _ = timed(lambda: [p.setup() for p in ps])
        single_setup.append(t)
        pb = [G.Plan.from_molecule(m, schwarz_thresh=1e-14).screen() for m in mols]
        t, _ = timed(lambda: G.setup_batch(pb))
        batch_setup.append(t)
        same_B = all(torch.equal(a.export(G.EXPORT_B), b.export(G.EXPORT_B)) for a, b in zip(ps, pb))
        for p in ps:
            p.close()
        if plans is not None:
            for p in plans:
                p.close()
        plans = pb
    noccs = [C.shape[1] for C in Cs]
    batch = G.Batch(plans, noccs)
    outs = [(torch.empty((p.nao, p.nao), dtype=torch.float64, device="cuda"),
             torch.empty((p.nao, p.nao), dtype=torch.float64, device="cuda"),
             torch.empty(2, dtype=torch.float64, device="cuda")) for p in plans]
    singles = [(torch.empty_like(o[0]), torch.empty_like(o[1]), torch.empty_like(o[2])) for o in outs]
    single_build, batch_build, graph_build = [], [], []
    for _ in range(reps + 1):   # the first pass warms up
        t, _ = timed(lambda: [p.build(C=C, out=o) for p, C, o in zip(plans, Cs, singles)])
        single_build.append(t)
        t, _ = timed(lambda: batch.build(Cs, outs=outs))
        batch_build.append(t)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.build(Cs, outs=outs)
    for _ in range(reps):
        t, _ = timed(g.replay)
        graph_build.append(t)
    dK = max(float((o[1] - q[1]).abs().max() / q[1].abs().max()) for o, q in zip(outs, singles))
    # the same in int8_fast (slices, grouped half transforms and int8 K)
    batch8 = G.Batch(plans, noccs, "int8_fast")
    single8, batched8 = [], []
    for _ in range(reps + 1):
        t, _ = timed(lambda: [p.build(C=C, precision="int8_fast", out=o) for p, C, o in zip(plans, Cs, singles)])
        single8.append(t)
        t, _ = timed(lambda: batch8.build(Cs, outs=outs))
        batched8.append(t)
    dK8 = max(float((o[1] - q[1]).abs().max() / q[1].abs().max()) for o, q in zip(outs, singles))
    for p in plans:
        p.close()
    return {"workload": "%d water clusters of 1-12 molecules (sizes %s), FP64" % (nmol, sizes),
            "nao_total": int(sum(m.nao for m in mols)),
            "setup_ms": {"one_by_one": round(min(single_setup), 2), "setup_batch": round(min(batch_setup), 2)},
            "setup_B_bitwise_equal": bool(same_B),
            "build_ms": {"one_by_one": round(min(single_build[1:]), 3), "build_batch": round(min(batch_build[1:]), 3),
                         "build_batch_graph_replay": round(min(graph_build), 3)},
            "max_rel_dK_batch_vs_single": dK,
            "build_ms_int8_fast": {"one_by_one": round(min(single8[1:]), 3), "build_batch": round(min(batched8[1:]), 3)},
            "max_rel_dK_batch_vs_single_int8_fast": dK8}


def make_inputs(n=32, box=10.0, geom_seed=1, cocc_seed=1):
    import workload as W
    z, x = W.water_cluster(n, box, geom_seed)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C0 = W.occupied_orbitals(S, mol.nelec // 2, cocc_seed)
    Cs = [W.perturbed_orbitals(C0, S, k, eps=1e-2, seed=1000) for k in range(NBUILDS)]
    return mol, S, Cs


def run_job(Plan, mol, Cd, precision, bufs, profile):
    """One job: setup + NBUILDS builds.  precision 'fp64' / 'int8' / 'int8_fast' / 'fp32' /
    'bf16x3' builds every K directly; '<p>_incr' builds K(C_0) in FP64 and
    each later K as K(C_0) + K(D - D_0) with the increment in precision <p>;
    'checked' runs dfjk_build_checked (int8 when its energy-error bound is
    within 1e-6 Eh, else FP64; 'checked_<budget>' another budget) and logs
    each build's choice and bound."""
    plan = Plan.from_molecule(mol, schwarz_thresh=1e-14)
    if profile:
        plan.profile(True)
    plan.screen().setup()
    outs = []
    incr = precision.endswith("_incr")
    base = precision[:-5] if incr else precision
    plan.checked_log = []
    for k, C in enumerate(Cd):
        J, K, E = bufs[k]
        if precision.startswith("checked"):
            budget = float(precision.split("_")[1]) if "_" in precision else 1e-6
            _, _, _, chosen, bound = plan.build_checked(C, budget=budget, out=(J, K, E))
            plan.checked_log.append((chosen, bound))
        elif incr and k > 0:
            plan.build_delta(C, Cd[0], bufs[0][1], precision=base, out=(J, K, E))
        else:
            plan.build(C=C, precision="fp64" if incr else base, out=(J, K, E))
        outs.append((J, K, E))
    return plan, outs


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(mol, Cs, target_s=20.0):
    """The FP64 oracle on a bounded sample of the same job, scaled to builds/s.

    Sample: (a) three-centre integrals for every 22nd aux shell (all AO pairs),
    scaled by the shell count; (b) the full metric; (c) the full Cholesky;
    (d) forward substitution of 16384 of the nao^2 pair columns, scaled;
    (e) one build's J and K over a slab of 64 aux functions, scaled by naux
    and by 10 builds."""
    import numpy as np
    import oracle
    t = {}
    nsh = len(mol.aux_l)
    pick = np.arange(0, nsh, 22)
    t0 = time.perf_counter()
    slabs = [oracle.int3c(mol, int(c), int(c) + 1) for c in pick]
    t["int3c"] = (time.perf_counter() - t0) * nsh / len(pick)
    t0 = time.perf_counter()
    V = oracle.int2c(mol)
    t["metric"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    L = oracle.cholesky(V)
    t["cholesky"] = time.perf_counter() - t0
    nao, naux = mol.nao, mol.naux
    rng = np.random.default_rng(0)
    U = np.concatenate([s.reshape(s.shape[0], -1) for s in slabs])
    ncol = 16384
    cols = rng.choice(nao * nao, size=ncol, replace=False)
    Ufull = np.zeros((naux, ncol))
    Ufull[: U.shape[0]] = U[:, cols]
    t0 = time.perf_counter()
    oracle.forward_subst(L, Ufull)
    t["whiten"] = (time.perf_counter() - t0) * (nao * nao) / ncol
    Bslab = np.concatenate(slabs)[:64]
    t0 = time.perf_counter()
    oracle.jk_from_B(Bslab, C=Cs[0])
    t["build"] = (time.perf_counter() - t0) * naux / Bslab.shape[0]
    total = t["int3c"] + t["metric"] + t["cholesky"] + t["whiten"] + NBUILDS * t["build"]
    return {
        "value": NBUILDS / total,
        "unit": "builds/s",
        "cores": int(oracle.num_threads()),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": ("water32 job (setup + 10 builds) timed on a sample: int3c for every 22nd aux shell "
                   "(x%.1f), full metric and Cholesky, forward substitution of %d of %d pair columns, "
                   "J/K of one build over %d of %d aux functions; each part scaled to the full job"
                   % (nsh / len(pick), ncol, nao * nao, Bslab.shape[0], naux)),
        "seconds_extrapolated": {k: round(v, 3) for k, v in t.items()},
        "job_seconds_extrapolated": round(total, 2),
    }


def serving_bench(modes, nreq, nmax, seed=3, max_active=4, budget_frac=0.6, loads=(0.8,)):
    """Continuous-batching serving of water clusters of 1..nmax molecules
    (NBUILDS SCF-like builds each): two closed-loop runs (every request queued
    at t = 0) give the saturation rate mu (their mean); then seeded Poisson streams at
    load x mu for each load give p50/p99 latency.  One molecule per size
    (geometry seed 10000 + n, box for the water32 density) serves every
    request of that size.  A mode is a precision ("fp64", "bf16x3_incr", ...),
    with "+batched" for the step-batched executor (grouped launches)."""
    import numpy as np
    import torch

    import workload as W
    from paper_2404_09452_amd.serve import (RUNTIME_RESERVE_BYTES, BatchedGpuExecutor, GpuExecutor, Request,
                                            Server, default_budget, summarize)
    _, sizes = W.poisson_stream(nreq, 1.0, seed, 1, nmax)
    pool = {}
    for n in sorted(set(int(s) for s in sizes)):
        z, x = W.water_cluster(n, W.cluster_box(n), 10000 + n) if n > 1 else W.water_monomer()
        mol = W.make_molecule(z, x)
        S = W.overlap_by_quadrature(mol)
        C0 = W.occupied_orbitals(S, mol.nelec // 2, n)
        pool[n] = (mol, [W.perturbed_orbitals(C0, S, k, eps=1e-2, seed=1000) for k in range(NBUILDS)])
    # the executors cap torch's allocator (serve.ALLOCATOR_FRACTION) and the
    # server keeps serve.RUNTIME_RESERVE_BYTES of the budget for the runtime
    GpuExecutor(keep_results=False)
    budget = default_budget(budget_frac)
    out = {"requests": nreq, "sizes": "uniform 1..%d waters" % nmax, "builds_per_request": NBUILDS,
           "max_active": max_active, "hbm_budget_GB": round(budget / 1e9, 1),
           "runtime_reserve_GB": round(RUNTIME_RESERVE_BYTES / 1e9, 1), "loads_x_saturation": list(loads)}
    for mode in modes:
        prec, batched = mode.split("+")[0], mode.endswith("+batched")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()            # each mode starts from the same allocator state

        def reqs(arrivals):
            return [Request(rid=i, mol=pool[int(n)][0], orbitals=pool[int(n)][1], arrival=float(a),
                            precision=prec) for i, (n, a) in enumerate(zip(sizes, arrivals))]

        def executor():
            return BatchedGpuExecutor(keep_results=False) if batched else GpuExecutor(keep_results=False)

        def progress(tag):
            count = [0]

            def done(req):
                count[0] += 1
                if count[0] % 16 == 0:
                    print("bench: serving %s %s: %d of %d requests done" % (mode, tag, count[0], nreq),
                          file=sys.stderr, flush=True)
            return done
        # an untimed pass first, so that the timed runs meet a warm allocator
        Server(executor(), max_active=max_active, hbm_budget_bytes=budget, runtime_reserve_bytes=RUNTIME_RESERVE_BYTES,
               on_done=progress("warm-up")).serve(reqs(np.zeros(nreq)))
        # two closed-loop passes (single passes of this mix move by tens of
        # percent); the saturation rate is their mean
        walls, sats, marks = [], [], []
        for rep in range(2):
            srv = Server(executor(), max_active=max_active, hbm_budget_bytes=budget,
                         runtime_reserve_bytes=RUNTIME_RESERVE_BYTES, on_done=progress("closed loop %d" % (rep + 1)))
            t0 = time.perf_counter()
            m0 = time.monotonic_ns()
            closed = srv.serve(reqs(np.zeros(nreq)))
            m1 = time.monotonic_ns()
            walls.append(time.perf_counter() - t0)
            sats.append(summarize(closed, walls[-1]))
            marks.append([m0, m1])
        wall = sum(walls) / len(walls)
        mu = nreq / wall
        failed = sum(st["failed"] for st in sats)
        print("bench: serving %s closed loop: %.2f req/s (passes %s), %d failed"
              % (mode, mu, " / ".join("%.2f" % (nreq / w) for w in walls), failed), file=sys.stderr, flush=True)
        r = {"saturation_requests_per_s": round(mu, 3),
             "saturation_requests_per_s_passes": [round(nreq / w, 3) for w in walls],
             "saturation_builds_per_s": round(sum(st["builds_per_s"] for st in sats) / len(sats), 2),
             "saturation_failed": failed, "closed_loop_monotonic_ns": marks}
        errors = [e for st in sats for e in st["errors"]]
        if errors:
            r["saturation_errors"] = errors
        for load in loads:
            arr, _ = W.poisson_stream(nreq, load * mu, seed, 1, nmax)
            srv = Server(executor(), max_active=max_active, hbm_budget_bytes=budget,
                         runtime_reserve_bytes=RUNTIME_RESERVE_BYTES, on_done=progress("load %.2f" % load))
            t0 = time.perf_counter()
            done = srv.serve(reqs(arr))
            wall = time.perf_counter() - t0
            st = summarize(done, wall)
            key = "" if len(loads) == 1 else "load_%.2f_" % load
            r.update({key + "poisson_rate_per_s": round(load * mu, 3),
                      key + "builds_per_s": round(st["builds_per_s"], 2),
                      key + "p50_latency_s": round(st["p50_latency_s"], 4),
                      key + "p99_latency_s": round(st["p99_latency_s"], 4),
                      key + "failed": st["failed"], key + "peak_active": srv.peak_active})
            if st["errors"]:
                r[key + "errors"] = st["errors"]
            print("bench: serving %s mu %.2f req/s, load %.2f: p50 %.3f s, p99 %.3f s" %
                  (mode, mu, load, st["p50_latency_s"], st["p99_latency_s"]), file=sys.stderr, flush=True)
        out[mode] = r
    return out


def large_setup_bench(nsetup):
    """`nsetup` setups of the 128-water cluster (the workload of large_bench):
    wall time and stage times of each."""
    import torch
    import workload as W
    from paper_2404_09452_amd.dfjk import Plan

    z, x = W.water_cluster(128, 16.0, 4)
    mol = W.make_molecule(z, x)
    runs = []
    for _ in range(nsetup):
        plan = Plan.from_molecule(mol, schwarz_thresh=1e-10).profile(True)
        plan.screen()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.setup()
        torch.cuda.synchronize()
        runs.append({"setup_s": round(time.perf_counter() - t0, 4),
                     "setup_stage_ms": {k: round(v[0], 3) for k, v in plan.profile_read().items()
                                        if k.startswith("setup.")}})
        print("bench: water128 setup %.4f s" % runs[-1]["setup_s"], file=sys.stderr, flush=True)
        del plan
        torch.cuda.empty_cache()
    return {"workload": "water128: 128-water cluster, 16 A box, 3840 AO / 11136 aux, Schwarz 1e-10", "runs": runs}


def large_bench(nbuild=2):
    """The 128-water cluster (3,840 AO, 11,136 aux, nocc 640, 16 A box, geometry
    seed 4, Schwarz 1e-10): one setup, then `nbuild` builds per precision with
    the K build streamed over aux slabs.  Reports ms per build, the K
    contraction's MFMA rate against each precision's peak, the integral and
    whitening times of the setup, and the energy error of the mixed builds
    (direct, and incremental from the first FP64 build) against FP64."""
    import numpy as np
    import torch
    import workload as W
    from paper_2404_09452_amd.dfjk import Plan

    z, x = W.water_cluster(128, 16.0, 4)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C0 = W.occupied_orbitals(S, mol.nelec // 2, 4)
    Cs = [torch.as_tensor(W.perturbed_orbitals(C0, S, k, eps=1e-2, seed=1000), device="cuda")
          for k in range(nbuild)]
    nao, naux, nocc = mol.nao, mol.naux, mol.nelec // 2
    plan = Plan.from_molecule(mol, schwarz_thresh=1e-10).profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.screen().setup()
    torch.cuda.synchronize()
    setup_wall = time.perf_counter() - t0
    st = plan.profile_read()
    info = plan.info()
    k_flops = float(nao) * (nao + 1) * naux * nocc
    out = {"workload": "water128: 128-water cluster, 16 A box, 3840 AO / 11136 aux / nocc 640, Schwarz 1e-10",
           "screening": {k: info[k] for k in ("sig_shell_pairs", "nshell_pairs", "nf", "triplets_kept")},
           "setup_s": round(setup_wall, 4),
           "setup_stage_ms": {k: round(v[0], 3) for k, v in st.items() if k.startswith("setup.")},
           "B_resident_GB": round(info["nf"] * info["naux_pad"] * 8 / 1e9, 2)}
    ref = None
    for prec, peak in (("fp64", PEAK_F64_TFLOPS), ("int8", PEAK_INT8_TOPS / I8_PRODUCTS),
                       ("int8_fast", PEAK_INT8_TOPS / I8F_PRODUCTS), ("fp32", PEAK_F32_TFLOPS),
                       ("bf16x3", PEAK_BF16_TFLOPS / 3.0), ("fp32_incr", PEAK_F32_TFLOPS)):
        incr = prec.endswith("_incr")
        Es = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, C in enumerate(Cs):
            if incr and k > 0:
                J, K, E = plan.build_delta(C, Cs[0], K0, precision="fp32")
            else:
                J, K, E = plan.build(C=C, precision="fp64" if incr else prec)
                if incr:
                    K0 = K
            Es.append(E)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = plan.profile_read()
        E = np.array([e.cpu().numpy() for e in Es])
        kms = st["build.K"][0] / max(nbuild - (1 if incr else 0), 1)
        r = {"ms_per_build": round(1000.0 * wall / nbuild, 2),
             "stage_ms_per_build": {k: round(v[0] / nbuild, 3) for k, v in st.items() if k.startswith("build.")},
             "E": E.tolist()}
        if not incr:
            r["K_tflops"] = round(k_flops / (kms * 1e-3) / 1e12, 2)
            r["K_frac_of_peak"] = round(k_flops / (kms * 1e-3) / 1e12 / peak, 4)
            if prec.startswith("int8"):
                r["K_int8_tops"] = round((I8_PRODUCTS if prec == "int8" else I8F_PRODUCTS) * k_flops
                                         / (kms * 1e-3) / 1e12, 1)
        if prec == "fp64":
            ref = E
        else:
            r["max_abs_dE_J"] = float(np.abs(E[:, 0] - ref[:, 0]).max())
            r["max_abs_dE_K"] = float(np.abs(E[:, 1] - ref[:, 1]).max())
            r["meets_1e-6_Eh"] = bool(max(r["max_abs_dE_J"], r["max_abs_dE_K"]) <= 1e-6)
        out[prec] = r
        plan._scratch = {}
        print("bench: water128 %s %.1f ms/build" % (prec, r["ms_per_build"]), file=sys.stderr, flush=True)
    # host-resident B (pinned memory, slabs streamed back during each build)
    plan.offload()
    torch.cuda.empty_cache()
    hb = {"B_host_GB": round(info["nf"] * info["naux_pad"] * 8 / 1e9, 2)}
    for prec in ("fp64", "int8", "fp32"):
        plan.build(C=Cs[0], precision=prec)
        torch.cuda.synchronize()
        plan.profile_read()
        t0 = time.perf_counter()
        for C in Cs:
            plan.build(C=C, precision=prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = plan.profile_read()
        hb[prec] = {"ms_per_build": round(1000.0 * wall / nbuild, 2),
                    "stage_ms_per_build": {k: round(v[0] / nbuild, 3) for k, v in st.items() if k.startswith("build.")}}
        plan._scratch = {}
        print("bench: water128 host-resident B %s %.1f ms/build" % (prec, hb[prec]["ms_per_build"]),
              file=sys.stderr, flush=True)
    out["host_resident_B"] = hb
    Eref = out["fp64"]["E"]
    plan.close()
    del plan
    torch.cuda.empty_cache()
    # setup straight into host memory under a device budget far below B:
    # U and B formed in row blocks, never whole in HBM
    budget = 6 << 30
    hplan = Plan.from_molecule(mol, schwarz_thresh=1e-10).profile(True).screen()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hplan.setup_host(max_device_bytes=budget)
    torch.cuda.synchronize()
    hs = {"device_budget_GB": round(budget / 1e9, 2),
          "device_workspace_GB": round(hplan.setup_host_info["device_bytes"] / 1e9, 3),
          "B_host_GB": round(hplan.setup_host_info["host_bytes"] / 1e9, 2),
          "setup_s": round(time.perf_counter() - t0, 4),
          "setup_stage_ms": {k: round(v[0], 3) for k, v in hplan.profile_read().items() if k.startswith("setup.")}}
    for prec in ("fp64", "int8"):
        Es = []
        hplan.build(C=Cs[0], precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for C in Cs:
            Es.append(hplan.build(C=C, precision=prec)[2])
        torch.cuda.synchronize()
        E = np.array([e.cpu().numpy() for e in Es])
        hs[prec] = {"ms_per_build": round(1000.0 * (time.perf_counter() - t0) / nbuild, 2),
                    "max_abs_dE_vs_device_fp64": float(np.abs(E - np.array(Eref)).max())}
        hplan._scratch = {}
    print("bench: water128 setup into host memory %.2f s (device workspace %.2f GB)"
          % (hs["setup_s"], hs["device_workspace_GB"]), file=sys.stderr, flush=True)
    out["setup_into_host_memory"] = hs
    hplan.close()
    torch.cuda.empty_cache()
    return out


def _mixed_summary(results):
    """The fastest mixed mode whose energies stay within 1e-6 Eh of the oracle
    on the water32 job, against the FP64 build of the same job."""
    f64 = results["fp64"]
    ok = {k: v for k, v in results.items() if k != "fp64" and v.get("meets_1e-6_Eh")}
    if not ok:
        return {"mode": None}
    k, v = max(ok.items(), key=lambda kv: kv[1]["builds_per_s"])
    return {"mode": k, "builds_per_s": round(v["builds_per_s"], 3), "fp64_builds_per_s": round(f64["builds_per_s"], 3),
            "speedup": round(v["builds_per_s"] / f64["builds_per_s"], 3),
            "ms_per_build": round(v["ms_per_build_steady"], 3), "fp64_ms_per_build": round(f64["ms_per_build_steady"], 3),
            "max_abs_dE_J_vs_oracle": v["max_abs_dE_J_vs_oracle"], "max_abs_dE_K_vs_oracle": v["max_abs_dE_K_vs_oracle"],
            "max_abs_dK_rows_vs_oracle": v["max_abs_dK_rows_vs_oracle"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--modes", default=None,
                    help="comma-separated water32 modes after fp64 (default: every mixed mode)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests per serving run (each load point and the closed loop)")
    ap.add_argument("--serve-max-waters", type=int, default=64)
    ap.add_argument("--no-large", action="store_true", help="skip the 128-water leg")
    ap.add_argument("--serve-modes", default="fp64,int8+batched,int8_fast+batched")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only run the serving stream: --serve-requests requests of 1..64 waters, Poisson "
                         "loads 0.5..1.1 x saturation, for each of --serve-modes; print its JSON")
    ap.add_argument("--serve-profile", action="store_true",
                    help="only the serving warm-up and closed-loop runs of --serve-modes with --serve-requests "
                         "requests of 1..64 waters (for a kernel trace); print their JSON")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the 128-water leg and print its JSON (for profiling)")
    ap.add_argument("--large-builds", type=int, default=2)
    ap.add_argument("--only-large-setup", type=int, default=0, metavar="N",
                    help="run only N setups of the 128-water cluster and print their stage times (for profiling "
                         "the integral kernels)")
    ap.add_argument("--no-direct", action="store_true", help="skip the four-centre direct J/K leg")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the batching leg (setup and builds of 16 uneven molecules)")
    ap.add_argument("--only-batching", action="store_true", help="run only the batching leg and print its JSON")
    ap.add_argument("--only-direct", action="store_true",
                    help="run only the four-centre direct J/K leg on the 32-water cluster and print its JSON")
    ap.add_argument("--direct-builds", type=int, default=5)
    ap.add_argument("--no-direct-incremental", action="store_true",
                    help="leave out the incremental direct builds (for counter runs of full builds only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (scales HBM byte counters)")
    args = ap.parse_args()
    # serving molecules of 1..64 waters needs unsplit large blocks (set before
    # torch touches the GPU; see serve.configure_allocator)
    if not args.no_serve or args.serve_sweep or args.serve_profile:
        from paper_2404_09452_amd.serve import configure_allocator
        configure_allocator()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "repeats": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the build would shard over aux slabs with one all-reduce of J and K).", file=sys.stderr)
        sys.exit(2)
    if args.serve_sweep:
        print(json.dumps({"serving_sweep": serving_bench(args.serve_modes.split(","), args.serve_requests, 64,
                                                         loads=(0.5, 0.75, 0.9, 1.1))}))
        return
    if args.serve_profile:
        print(json.dumps({"serving_profile": serving_bench(args.serve_modes.split(","), args.serve_requests, 64,
                                                           loads=())}))
        return
    if args.only_large_setup:
        print(json.dumps({"water128_setup": large_setup_bench(args.only_large_setup)}))
        return
    if args.only_batching:
        print(json.dumps({"batching": batching_bench()}))
        return
    if args.only_large:
        print(json.dumps({"water128": large_bench(args.large_builds)}))
        return
    if args.only_direct:
        import torch
        mol, S, Cs = make_inputs()
        Cd = [torch.as_tensor(C, device="cuda") for C in Cs]
        print(json.dumps({"direct_scf": direct_bench(mol, Cd, nbuild=args.direct_builds,
                                                     S=None if args.no_direct_incremental else S)}))
        return
    import numpy as np
    import torch
    from paper_2404_09452_amd.dfjk import Plan

    dev = torch.device("cuda")
    print("bench: building inputs (32-water cluster)", file=sys.stderr, flush=True)
    mol, S, Cs = make_inputs()
    Cd = [torch.as_tensor(C, device=dev) for C in Cs]
    nao = mol.nao
    bufs = [(torch.empty((nao, nao), dtype=torch.float64, device=dev),
             torch.empty((nao, nao), dtype=torch.float64, device=dev),
             torch.empty(2, dtype=torch.float64, device=dev)) for _ in range(NBUILDS)]

    results = {}
    ref_E = None
    ref_K = None
    modes = ["fp64"] + ([] if args.no_mixed else ["int8", "int8_fast", "checked", "checked_1e-5", "fp32", "bf16x3",
                                                      "fp32_incr", "bf16x3_incr"])
    if args.modes:
        modes = ["fp64"] + [m for m in args.modes.split(",") if m != "fp64"]
    for prec in modes:
        for w in range(args.warmup):
            run_job(Plan, mol, Cd, prec, bufs, profile=False)
        torch.cuda.synchronize()
        print("bench: timing %d steps, %s" % (args.steps, prec), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        stage_ms, stage_n = {}, {}
        step_ms = []
        for s in range(args.steps):
            ts = time.perf_counter()
            plan, outs = run_job(Plan, mol, Cd, prec, bufs, profile=True)
            torch.cuda.synchronize()
            step_ms.append(1000.0 * (time.perf_counter() - ts))
            for k, (ms, n) in plan.profile_read().items():
                stage_ms[k] = stage_ms.get(k, 0.0) + ms
                stage_n[k] = stage_n.get(k, 0) + n
            info = plan.info()
            checked_log = plan.checked_log
            plan.close()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        E = np.array([o[2].cpu().numpy() for o in outs])
        K_last = outs[-1][1].cpu().numpy()
        setup_ms = (stage_ms["span.setup"] if stage_n.get("span.setup") else
                    sum(stage_ms[k] for k in stage_ms if k.startswith("setup."))) / args.steps
        # a build's span on its stream (J overlaps the half transform and K on a
        # side stream, so the stage times overlap); the stage sum where a mode
        # records no span
        build_ms = (stage_ms["span.build"] if stage_n.get("span.build") else
                    sum(stage_ms[k] for k in stage_ms if k.startswith("build."))) / (args.steps * NBUILDS)
        r = {
            "builds_per_s": NBUILDS * args.steps / dt,
            "ms_per_step": 1000.0 * dt / args.steps,
            "ms_per_step_median": float(np.median(step_ms)),
            "ms_per_step_min": float(np.min(step_ms)),
            "ms_per_build_steady": build_ms,
            "setup_ms": setup_ms,
            "stages_ms_per_launch": {k: round(stage_ms[k] / max(stage_n[k], 1), 4) for k in stage_ms},
            "stage_launches": stage_n,
            "E_J": E[:, 0].tolist(),
            "E_K": E[:, 1].tolist(),
        }
        r.update(golden_errors(E, K_last))
        if prec.startswith("checked"):
            r["per_build_choice"] = [c for c, _ in checked_log]
            r["per_build_bound_Eh"] = [float("%.4g" % b) for _, b in checked_log]
        if prec == "fp64":
            ref_E, ref_K = E, K_last
            r["screening"] = {k: info[k] for k in ("sig_shell_pairs", "nshell_pairs", "nf", "triplets_kept")}
        else:
            r["max_abs_dE_J_vs_fp64"] = float(np.abs(E[:, 0] - ref_E[:, 0]).max())
            r["max_abs_dE_K_vs_fp64"] = float(np.abs(E[:, 1] - ref_E[:, 1]).max())
            r["max_abs_dK_vs_fp64"] = float(np.abs(K_last - ref_K).max())
            r["meets_1e-6_Eh"] = bool(max(r["max_abs_dE_J_vs_oracle"], r["max_abs_dE_K_vs_oracle"]) <= 1e-6)
        results[prec] = r
        print("bench: %s %.2f builds/s, %.3f ms/build steady, setup %.1f ms" %
              (prec, r["builds_per_s"], build_ms, setup_ms), file=sys.stderr, flush=True)

    f64 = results["fp64"]
    naux, nocc = mol.naux, mol.nelec // 2
    # the FP64 build's K launch shape (tile, split count) before any autotuning
    tplan = Plan.from_molecule(mol, schwarz_thresh=1e-14).screen()
    shape = tplan.build_shape(nocc)
    k_flops = float(nao) * (nao + 1) * naux * nocc        # lower triangle of 2 X X^T per build, useful flops
    # the K contraction of a build runs as one launch per aux slab (equal slabs
    # here); per launch: the build's flops over the launches, the mean duration
    k_launches = f64["stage_launches"]["build.K"] / (args.steps * NBUILDS)
    k_ms = f64["stages_ms_per_launch"]["build.K"]
    achieved = k_flops / k_launches / (k_ms * 1e-3) / 1e12
    roofline = {"kernel": "build.K (FP64 MFMA X X^T, k_syrk_f64<%d>, %d splits)" % (shape["k_tile"], shape["nsplit"]),
                "bound": "mfma",
                "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_F64_TFLOPS, 4), "traffic": committed_traffic(shape),
                "traffic_source": "profiles/k_syrk_f64_water32.md (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, per launch)",
                "flops_per_launch": k_flops / k_launches, "ms_per_launch": k_ms, "launches_per_build": k_launches}
    # the other steps of an FP64 build against their bounds (HIP-event stage times;
    # algorithmic bytes: J reads B twice, the half transform reads B twice and
    # writes X once)
    scr = f64["screening"]
    nf, npad = scr["nf"], -(-naux // 128) * 128
    b_bytes = float(nf) * npad * 8
    j_ms = f64["stages_ms_per_launch"]["build.J"]
    ht_ms = f64["stages_ms_per_launch"]["build.halftransform"]
    ht_bytes = 2 * b_bytes + float(nao) * npad * nocc * 8
    by_step = {
        "J": {"bound": "hbm", "bytes": 2 * b_bytes, "ms": j_ms,
              "GB_per_s": round(2 * b_bytes / (j_ms * 1e-3) / 1e9, 1),
              "frac": round(2 * b_bytes / (j_ms * 1e-3) / PEAK_HBM_BYTES, 4)},
        "halftransform": {"bound": "hbm", "bytes": ht_bytes, "ms": ht_ms,
                          "GB_per_s": round(ht_bytes / (ht_ms * 1e-3) / 1e9, 1),
                          "frac": round(ht_bytes / (ht_ms * 1e-3) / PEAK_HBM_BYTES, 4)},
        "K": {"bound": "mfma", "frac": roofline["frac"]},
        "int3c": {"bound": "fp64 valu", "ms_per_setup": f64["stages_ms_per_launch"].get("setup.int3c"),
                  "shell_triplets": scr["triplets_kept"],
                  "note": "FP64 VALU fraction from counters: profiles/int3c_water128.md"},
    }
    for prec, peak in (("int8", PEAK_INT8_TOPS / I8_PRODUCTS), ("int8_fast", PEAK_INT8_TOPS / I8F_PRODUCTS),
                       ("fp32", PEAK_F32_TFLOPS),
                       ("bf16x3", PEAK_BF16_TFLOPS / 3.0)):
        if prec in results:
            n_l = results[prec]["stage_launches"]["build.K"] / (args.steps * NBUILDS)
            ms = results[prec]["stages_ms_per_launch"]["build.K"] * n_l        # per build
            results[prec]["K_tflops"] = round(k_flops / (ms * 1e-3) / 1e12, 2)
            results[prec]["K_frac_of_peak"] = round(k_flops / (ms * 1e-3) / 1e12 / peak, 4)
            if prec.startswith("int8"):
                results[prec]["K_int8_tops"] = round((I8_PRODUCTS if prec == "int8" else I8F_PRODUCTS) * k_flops
                                                     / (ms * 1e-3) / 1e12, 1)

    direct = None
    if not args.no_direct:
        print("bench: four-centre direct J/K", file=sys.stderr, flush=True)
        direct = direct_bench(mol, Cd, nbuild=args.direct_builds, E_df=ref_E, S=S)

    batching = None
    if not args.no_batching:
        print("bench: batching of uneven molecules", file=sys.stderr, flush=True)
        batching = batching_bench()

    # split-count autotuner on the same molecule (outside the timed steps)
    tplan.setup()
    chosen, cand_ms = tplan.autotune(Cd[0])
    autotune = {"chosen_tile": chosen[0], "chosen_nsplit": chosen[1],
                "ms_per_build_by_tile_and_nsplit": {"%dx%d" % k: round(v, 3) for k, v in cand_ms.items()}}
    tplan.close()
    del bufs, Cd
    torch.cuda.empty_cache()
    large = None
    if not args.no_large:
        print("bench: 128-water cluster", file=sys.stderr, flush=True)
        large = large_bench(args.large_builds)

    serving = None
    if not args.no_serve:
        print("bench: serving stream", file=sys.stderr, flush=True)
        serving = serving_bench(args.serve_modes.split(","), args.serve_requests, args.serve_max_waters,
                                loads=(0.5, 0.9, 1.1))

    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(mol, Cs)

    line = {
        "metric": "DF-J/K builds/sec + ms per build (FP64 vs mixed, |dE|<=1e-6 Eh); p99 serve latency",
        "value": round(f64["builds_per_s"], 3),
        "unit": "builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 3),
        "ms_per_step_median": round(f64["ms_per_step_median"], 3),
        "ms_per_step_min": round(f64["ms_per_step_min"], 3),
        "ms_per_build": round(f64["ms_per_build_steady"], 3),
        "setup_ms": round(f64["setup_ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "water32: 32-water cluster, 960 AO / 2784 aux / nocc 160, "
                               "Schwarz 1e-14, setup + 10 builds per step",
                   "nao": nao, "naux": naux, "nocc": nocc, "builds_per_step": NBUILDS},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": {k: v for k, v in results.items() if k != "fp64"},
        "mixed_vs_fp64": _mixed_summary(results),
        "serving": serving,
        "water128": large,
        "direct_scf": direct,
        "batching": batching,
        "autotune_K_split": autotune,
        "roofline_by_step": by_step,
        "fp64_detail": {k: v for k, v in f64.items() if k not in ("E_J", "E_K")},
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
