"""Benchmark of the hot path on one MI355X.

One step = one stencil setup (shift list, Green's sums, Gram + null vectors,
per-point P rows) followed by one pseudospectral apply (L + diag v) u, on the
2D Helmholtz workload with n = 1024 (N = 1,048,576 points), t = 2 (5x5
stencils), |S| = 64, FP64. Inputs are resident on the GPU before timing.

Prints one JSON line. value = local stencils per second, N / (mean device
time of one setup over max(K, 100) setups after W of their own, two events on
the stream: a steady-state rate; the same count times the apply, the C-apply
and the other setup forms of this workload). ms_per_step is
the wall time of the K timed steps (setup + apply) between device
synchronisations. ps_apply bandwidth is algorithmic bytes / mean apply time.
The roofline of the dominant kernel (the per-point assembly) uses its average
duration from per-stage HIP events that the library records on its stream.

A second section compares the learned-stencil setup (a BF16 surrogate network
beside the method, with exact fallback) with the exact setup on the 3D
Helmholtz workload n = 64, t = 1, |S| = 16: the network is trained on the GPU
on 200,000 exact rows of other fields (seeds 1..8), both setups are timed on
the evaluation field (seed 0), and GMRES(40) iteration counts to 1e-8 are
compared on the same kind of field at n = 16, where the host LU of P is cheap,
with a network trained the same way on n = 16 fields (its fallback fraction is
reported beside the counts).

A Krylov section runs GMRES(40) with every step on the device (the P-solve
with nested-dissection factors of P computed on the host) on the 2D
cross-profile field at n = 256, and times one Arnoldi step, graph-replayed
and launched directly, and the P-solve alone.

A third section times the batched form: 64 2D problems with n drawn from
{64, 128, 256, 512}, set up (FP32 rows) and applied with one launch per stage
for all of them, against the same 64 problems set up one by one.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--no-learned] [--train-steps S] [--no-batched] [--no-extras]
    python bench.py --krylov-only      # the device-GMRES section alone
    python bench.py --copy-probe MiB   # plain device copy of a known size, for
                                       # scaling hardware byte counters
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "local stencils/s + ps_apply GB/s, 2D n=1024; learned vs exact at equal GMRES iters"
HBM_PEAK_GBPS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 MFMA

# HBM bytes per launch of the assembly kernel on this workload, from the
# FETCH_SIZE and WRITE_SIZE hardware counters (rocprofv3 --pmc, one counter
# per run), each scaled by what the same counter reads for a plain 256 MiB
# device copy (FETCH_SIZE reads half of the copied bytes: scale 2.000;
# WRITE_SIZE all of them: scale 1.000). The readings hold for the kernel
# sources they were taken on (sha256 prefix of the files below); for any
# other sources the traffic is reported as null.
ASSEMBLE_PMC = {
    "fetch_kib": 5283.7, "write_kib": 208931.8,
    "fetch_scale": 262144.0 / 131093.4, "write_scale": 262144.0 / 262144.0,
    "sources": ("paper_1607_02560_amd/csrc/assemble.hip",
                "paper_1607_02560_amd/csrc/setup_common.h"),
    "sources_sha256": "aec2d058f06f6800",
}


def assemble_traffic():
    """Counter-based HBM bytes per assembly launch, or None if the kernel
    sources differ from those the counters were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ASSEMBLE_PMC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != ASSEMBLE_PMC["sources_sha256"]:
        return None
    return (ASSEMBLE_PMC["fetch_kib"] * ASSEMBLE_PMC["fetch_scale"]
            + ASSEMBLE_PMC["write_kib"] * ASSEMBLE_PMC["write_scale"]) * 1024.0


def algorithmic_bytes(N, m):
    """Minimum HBM traffic per call (see the design notes):
    setup reads v (8 B/pt) and writes P (8 m B/pt) and idx (4 B/pt);
    ps_apply reads u (16 B) and v (8 B) and writes y (16 B) per point;
    the C-apply reads r (16 B) and v (8 B, for the point's shift) and writes
    z (16 B) per point."""
    return {"assemble": N * (8 + 8 * m + 4), "setup": N * (8 + 8 * m + 4), "apply": N * 40,
            "c_apply": N * 40}


def timed(stream, fn, reps):
    """Mean device time of fn over reps calls, two events on the stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def learned_vs_exact(dev, stream, reps, train_steps, threshold=1e-3):
    """The learned-stencil setup against the exact setup (3D Helmholtz, t = 1)."""
    import numpy as np
    import torch
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import surrogate as SG
    from paper_1607_02560_amd import workloads as W
    n, t, nS, batch = 64, 1, 16, 8192
    m = (2 * t + 1) ** 3
    print("[bench] learned: gathering 200k exact training rows (seeds 1..8)", file=sys.stderr,
          flush=True)
    fields = [W.helm3d_random(n, seed=s).v for s in range(1, 9)]
    t0 = time.perf_counter()
    X, T = SG.gather_rows(fields, t, nS, 25000, seed=100, device=dev)
    torch.cuda.synchronize()
    t_gather = time.perf_counter() - t0
    net = SG.make_mlp(3, t, seed=101, batch_rows=batch)
    net.fit_normalisation(X, T)
    print(f"[bench] learned: training {train_steps} Adam steps of {batch} rows", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    hist = SG.train(net, X, T, train_steps, batch, 3e-3, seed=102,
                    report_every=max(train_steps // 4, 1), lr_final=2e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    N = n ** 3
    ev = W.helm3d_random(n, seed=0)
    prob = lsp.Problem(3, n, torch.from_numpy(ev.v.reshape(-1)).to(dev))
    P = torch.empty(N * m, dtype=torch.float64, device=dev)
    idx = torch.empty(N, dtype=torch.int32, device=dev)
    fb = torch.empty(N, dtype=torch.int32, device=dev)
    exact = lambda: prob.stencil_setup(t, nS, P, idx)
    # asynchronous calls, like the exact setup; the count is read afterwards
    learned = lambda: prob.stencil_setup_learned(net, t, nS, threshold, P, fb, count=False)
    for _ in range(3):
        exact()
        learned()
    t_exact = timed(stream, exact, reps)
    t_learned = timed(stream, learned, reps)
    # the network-and-rows kernel alone (per-stage HIP events of the library)
    prob.profile(True)
    for _ in range(reps):
        learned()
    prof = prob.profile_read()
    prob.profile(False)
    t_rows = prof["assemble"][0] / max(prof["assemble"][1], 1) * 1e-3
    nf = [prob.stencil_setup_learned(net, t, nS, threshold, P, fb)]
    prob.close()
    net.close()
    # GMRES(40) to 1e-8 on an n = 16 field of the same kind (seed 0), where the
    # host LU of P is cheap, with a network trained the same way on n = 16
    # fields (seeds 1..8, every point): the comparison runs with the network's
    # rows, and the fallback fraction says how many
    print("[bench] learned: GMRES comparison at n=16", file=sys.stderr, flush=True)
    ns = 16
    Xs, Ts = SG.gather_rows([W.helm3d_random(ns, seed=s).v for s in range(1, 9)], t, 0, ns ** 3,
                            seed=103, device=dev)
    net16 = SG.make_mlp(3, t, seed=104, batch_rows=4096)
    net16.fit_normalisation(Xs, Ts)
    SG.train(net16, Xs, Ts, 2000, 4096, 3e-3, seed=105, lr_final=3e-4)
    small = W.helm3d_random(ns, seed=0)
    Ns = ns ** 3
    probs = lsp.Problem(3, ns, torch.from_numpy(small.v.reshape(-1)).to(dev))
    ft = torch.from_numpy(small.f.reshape(-1)).to(dev)
    Ps = torch.empty(Ns * m, dtype=torch.float64, device=dev)
    fbs = torch.empty(Ns, dtype=torch.int32, device=dev)
    gm = {"network": f"trained on {int(Xs.shape[0])} exact rows of n={ns} fields (seeds 1..8), "
                     f"2000 Adam steps of 4096 rows", "threshold_excess": threshold}
    for name in ("exact", "learned"):
        if name == "exact":
            probs.stencil_setup(t, small.num_shifts, Ps)
            nfs = 0
        else:
            nfs = probs.stencil_setup_learned(net16, t, small.num_shifts, threshold, Ps, fbs)
        solve = lsp.host_lu_solver(Ps.cpu().numpy().reshape(Ns, m), 3, ns, t)
        ut = torch.zeros_like(ft)
        code, iters, relres = probs.precond_solve(ft, ut, solve, rtol=1e-8, restart=40, maxit=400)
        gm[name] = {"iterations": iters, "relres": relres, "status": code, "fallback_rows": nfs,
                    "fallback_frac": nfs / Ns}
    probs.close()
    net16.close()
    # MFMA work: BF16 products of the network (unpadded sizes), against the
    # dense BF16 peak of the part
    n_in, n_h, n_out = m + 2, SG.HIDDEN, 2 * m
    fwd = 2 * (n_in * n_h + n_h * n_h + n_h * n_out)            # flop per row, forward
    train = fwd + fwd + 2 * (n_h * n_h + n_out * n_h)           # + weight and input gradients
    sps = train_steps * batch / t_train
    return {
        "workload": f"3D Helmholtz, smooth random c in [0.8,1.2], n={n} (N={N}), t={t} "
                    f"(3x3x3 stencils), |S|={nS}, evaluation seed 0",
        "mfma": {"peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "flop_per_row_forward": fwd, "flop_per_row_train": train,
                 "train_achieved": sps * train / 1e12,
                 "train_frac": sps * train / 1e12 / BF16_PEAK_TFLOPS,
                 "learned_rows_kernel_ms": t_rows * 1e3,
                 "learned_rows_achieved": N * fwd / t_rows / 1e12,
                 "learned_rows_frac": N * fwd / t_rows / 1e12 / BF16_PEAK_TFLOPS},
        "network": f"{m + 2}->{SG.HIDDEN}->{SG.HIDDEN}->{2 * m} SiLU, BF16 MFMA, FP32 accumulation",
        "training": {"rows": int(X.shape[0]), "seeds": "1..8", "steps": train_steps,
                     "batch": batch, "loss_by_step": [[int(a), float(b)] for a, b in hist],
                     "gather_s": t_gather, "train_s": t_train,
                     "samples_per_s": train_steps * batch / t_train},
        "threshold_excess": threshold,
        "exact_setup_ms": t_exact * 1e3,
        "learned_setup_ms": t_learned * 1e3,
        "learned_over_exact_time": t_learned / t_exact,
        "fallback_rows": nf[0], "fallback_frac": nf[0] / N,
        "gmres_n16": gm,
        "gmres_iterations_equal_within_1": abs(gm["exact"]["iterations"]
                                               - gm["learned"]["iterations"]) <= 1,
    }


def batched_section(dev, reps):
    """The batched form on 64 problems of uneven n (2D Helmholtz, t = 2,
    |S_p| = n_p / 16, FP32 rows): batched setup and apply (graph replays)
    against the same 64 single-problem calls back to back."""
    import torch
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import workloads as W
    print("[bench] batched: 64 problems", file=sys.stderr, flush=True)
    ps = W.batch2d(64, seed=0)
    stream = torch.cuda.Stream(dev)
    probs = [lsp.Problem(2, p.n, torch.from_numpy(p.v.reshape(-1)).to(dev), stream=stream)
             for p in ps]
    m = 25
    Ps = [torch.empty(p.N * m, dtype=torch.float32, device=dev) for p in ps]
    idxs = [torch.empty(p.N, dtype=torch.int32, device=dev) for p in ps]
    us = [torch.from_numpy(p.f.reshape(-1)).to(dev) for p in ps]
    ys = [torch.empty_like(u) for u in us]
    nS = [p.num_shifts for p in ps]
    torch.cuda.synchronize()
    batch = lsp.Batch(probs)
    bsetup = lambda: batch.stencil_setup(2, nS, Ps, idxs, precision=lsp.LSP_FP32_REFINE)
    bapply = lambda: batch.ps_apply(us, ys)

    def singles_setup():
        for i, pr in enumerate(probs):
            pr.stencil_setup(2, nS[i], Ps[i], idxs[i], precision=lsp.LSP_FP32_REFINE)

    def singles_apply():
        for i, pr in enumerate(probs):
            pr.ps_apply(us[i], ys[i])

    for fn in (bsetup, bapply, singles_setup, singles_apply):
        for _ in range(3):
            fn()
    t_bs = timed(stream, bsetup, reps)
    t_ba = timed(stream, bapply, reps)
    t_ss = timed(stream, singles_setup, reps)
    t_sa = timed(stream, singles_apply, reps)
    tw, cand, ms = batch.tile()
    total = sum(p.N for p in ps)
    batch.close()
    for pr in probs:
        pr.close()
    return {
        "workload": "64 x 2D Helmholtz, n drawn from {64,128,256,512} (seed 0), own smooth "
                    "random c in [0.8,1.2] each, t=2 (5x5 stencils), |S_p|=n_p/16, FP32 rows",
        "sizes": {str(n): sum(1 for p in ps if p.n == n) for n in (64, 128, 256, 512)},
        "points": total,
        "batched_setup_ms": t_bs * 1e3, "batched_stencils_per_s": total / t_bs,
        "single_setups_ms": t_ss * 1e3, "single_stencils_per_s": total / t_ss,
        "batched_apply_ms": t_ba * 1e3, "single_applies_ms": t_sa * 1e3,
        "tile_width": tw, "tile_candidates": cand, "tile_candidate_ms": ms,
    }


def _oracle_tables_worker(args):
    """One process of the all-cores oracle timing: the oracle's per-shift
    tables (Green's kernels by FFT, Gram matrix, null vector) for a slice of
    the shift list."""
    d, n, S, t = args
    from oracle import lsp_oracle as O
    tab = O.shift_tables(d, n, S, t)
    return tab["alpha"], tab["C"]


def _oracle_apply_worker(args):
    """One process of the all-cores oracle timing: `reps` oracle applies."""
    v, f, reps = args
    from oracle import lsp_oracle as O
    t0 = time.perf_counter()
    for _ in range(reps):
        O.ps_apply(v, f)
    return time.perf_counter() - t0


def cpu_baseline(p):
    """The FP64 oracle timed on this host: one full setup of the same workload
    (the sample) and 10 applies, on one core (numpy's FFT is single-threaded)
    and on all cores. On all cores the oracle's functions run unchanged in
    one process per core: the per-shift tables (independent per shift) are
    split over the processes and the shift list, assignment and rows run in
    the parent; for the apply every process runs the oracle's apply, and the
    rate is the applies all processes complete per second."""
    import multiprocessing as mp

    import numpy as np
    from oracle import lsp_oracle as O
    t0 = time.perf_counter()
    O.stencil_setup(p.v, p.t, p.num_shifts)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        O.ps_apply(p.v, p.f)
    t_apply = (time.perf_counter() - t0) / reps
    out = {
        "value": p.N / t_setup, "unit": "stencils/s", "cores": 1, "kind": "oracle",
        "sample": f"one full setup of the same workload (N={p.N}, |S|={p.num_shifts}) "
                  f"and {reps} applies; numpy FFT single-threaded",
        "setup_s": t_setup, "ps_apply_s": t_apply,
        "ps_apply_GBps": 40.0 * p.N / t_apply / 1e9,
        "host_cpus": os.cpu_count(),
    }
    # all cores: at most 16 processes (the host share of one GPU on the
    # benchmark machines), spawned (not forked: the parent holds the GPU)
    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_tables_worker, [(p.d, 8, np.asarray([-1e3]), 1)] * workers)  # warm-up
        t0 = time.perf_counter()
        S = O.shift_list(p.v, p.num_shifts)
        parts = pool.map(_oracle_tables_worker,
                         [(p.d, p.n, S[i::workers], p.t) for i in range(workers)
                          if len(S[i::workers])])
        m = (2 * p.t + 1) ** p.d
        alpha = np.zeros((len(S), m))
        C = np.zeros((len(S), m))
        for i, (a, c) in enumerate(parts):
            alpha[i::workers] = a
            C[i::workers] = c
        idx = O.assign_shifts(p.v, S)
        O.assemble(p.v, S, alpha, C, idx, O.offsets(p.d, p.t))
        t_setup_all = time.perf_counter() - t0
        t0 = time.perf_counter()
        pool.map(_oracle_apply_worker, [(p.v, p.f, reps)] * workers)
        t_apply_all = (time.perf_counter() - t0) / (reps * workers)
        # let the workers exit by themselves before the pool is torn down, so
        # that no process outlives the benchmark
        pool.close()
        pool.join()
    # the spawn context also started multiprocessing's resource-tracker
    # process, which otherwise lives until this interpreter exits: release the
    # pool's semaphores first (collecting the pool unregisters them), then stop
    # the tracker and wait for it
    import gc
    from multiprocessing import resource_tracker
    del pool
    gc.collect()
    tracker = getattr(resource_tracker, "_resource_tracker", None)
    if tracker is not None and hasattr(tracker, "_stop"):
        tracker._stop()
    out["all_cores"] = {
        "cores": workers, "value": p.N / t_setup_all, "unit": "stencils/s",
        "setup_s": t_setup_all, "ps_apply_s_per_apply": t_apply_all,
        "ps_apply_GBps": 40.0 * p.N / t_apply_all / 1e9,
        "sample": f"the same setup with the per-shift tables split over {workers} processes; "
                  f"{reps} applies in each of {workers} processes",
    }
    return out


def non_localized_section(dev, t_setup_g, N):
    """The one-shift method of Sec. 3 beside the localized one: its setup
    time on the benchmark's field, and GMRES(40) iteration counts of both
    preconditioners on two smaller fields of Sec. 5's families (host LU of P)."""
    import torch
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import workloads as W
    out = {"setup_ms": t_setup_g * 1e3, "stencils_per_s": N / t_setup_g, "gmres": {}}
    for q in (W.helm2d_gauss(128), W.helm2d_cross(256)):
        Nq, mq = q.N, (2 * q.t + 1) ** q.d
        pr = lsp.Problem(q.d, q.n, torch.from_numpy(q.v.reshape(-1)).to(dev))
        ft = torch.from_numpy(q.f.reshape(-1)).to(dev)
        Pq = torch.empty(Nq * mq, dtype=torch.float64, device=dev)
        gm = {"workload": f"{q.name}, n={q.n}, t={q.t}, |S|={q.num_shifts} (localized)"}
        for name in ("localized", "non_localized"):
            if name == "localized":
                pr.stencil_setup(q.t, q.num_shifts, Pq)
            else:
                pr.stencil_setup_global(q.t, Pq)
            S = pr.get_tables()["S"]
            solve = lsp.host_lu_solver(Pq.cpu().numpy().reshape(Nq, mq), q.d, q.n, q.t)
            ut = torch.zeros_like(ft)
            code, iters, relres = pr.precond_solve(ft, ut, solve, rtol=1e-8, restart=40,
                                                   maxit=400)
            gm[name] = {"iterations": iters, "relres": relres, "status": code,
                        "shifts": len(S)}
        pr.close()
        out["gmres"][f"{q.name}_n{q.n}"] = gm
    return out


def krylov_section(dev, reps):
    """GMRES(40) with every step on the device (eq. (PC), Sec. 5), on the 2D
    cross-profile Helmholtz field at n = 256: P rows of the uniform t = 1
    setup and of the per-point radius (leaf box 8, t <= 2), factorised on the
    host by nested dissection (Sec. 3, Fig. 1) and solved on the device. One
    Arnoldi step (C-apply, P-solve, ps_apply, two Gram-Schmidt passes,
    Givens) is timed with HIP events around each step, replayed from its
    captured graph and launched directly; the P-solve alone is timed too."""
    import numpy as np
    import scipy.sparse
    import torch
    from paper_1607_02560_amd import lsp, nd
    from paper_1607_02560_amd import workloads as W
    q = W.helm2d_cross(256)
    out = {"workload": f"{q.name}, n={q.n} (N={q.N}), |S|={q.num_shifts}, rtol 1e-8, "
                       "restart 40", "cases": {}}
    stream = torch.cuda.Stream(dev)
    ft = torch.from_numpy(q.f.reshape(-1)).to(dev)
    for label, t, leaf in (("t1", 1, None), ("nd_radius_leaf8", 2, 8)):
        m = (2 * t + 1) ** 2
        res = {}
        for graphs in ("1", "0"):
            old = os.environ.get("LSP_GRAPHS")
            os.environ["LSP_GRAPHS"] = graphs
            try:
                pr = lsp.Problem(2, q.n, torch.from_numpy(q.v.reshape(-1)).to(dev),
                                 stream=stream)
            finally:
                if old is None:
                    os.environ.pop("LSP_GRAPHS", None)
                else:
                    os.environ["LSP_GRAPHS"] = old
            Pq = torch.empty(q.N * m, dtype=torch.float64, device=dev)
            if leaf:
                pr.stencil_setup_nd(leaf, q.num_shifts, Pq)
            else:
                pr.stencil_setup(t, q.num_shifts, Pq)
            torch.cuda.synchronize()
            rows = Pq.cpu().numpy().reshape(q.N, m)
            cols = lsp.export_pattern(2, q.n, t)
            S = scipy.sparse.csr_matrix((rows.reshape(-1), cols.reshape(-1),
                                         np.arange(0, q.N * m + 1, m)), shape=(q.N, q.N))
            t0 = time.perf_counter()
            F = nd.factor(S, 2, q.n, leaf or 8)
            t_factor = time.perf_counter() - t0
            ex = F.export()
            t0 = time.perf_counter()
            pr.psolve_upload(ex)
            t_upload = time.perf_counter() - t0
            ut = torch.zeros_like(ft)
            pr.precond_solve_device(ft, ut, rtol=1e-8, restart=40, maxit=400)  # capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, iters, relres = pr.precond_solve_device(ft, ut, rtol=1e-8, restart=40,
                                                          maxit=400)
            t_solve = time.perf_counter() - t0
            pr.profile(True)
            pr.precond_solve_device(ft, ut, rtol=1e-8, restart=40, maxit=400)
            rt = torch.from_numpy(q.f.reshape(-1)).to(dev)
            zt = torch.empty_like(rt)
            for _ in range(reps):
                pr.psolve_apply(rt, zt)
            prof = pr.profile_read()
            pr.profile(False)
            step_ms = prof["arnoldi"][0] / max(prof["arnoldi"][1], 1)
            ps_ms = prof["psolve"][0] / max(prof["psolve"][1], 1)
            entry = {"iterations": iters, "relres": relres, "status": code,
                     "solve_ms": t_solve * 1e3, "arnoldi_step_ms": step_ms}
            if graphs == "1":
                # algorithmic bytes of one P-solve: every dense block read
                # once, r read, z written, the index lists and the update
                # slots read (solve buffers are reread per level: not counted)
                nb = 8 * ex["data"].size + 32 * q.N + 8 * (3 * q.N + 2 * ex["idx_U"].size)
                entry.update({
                    "host_factor_s": t_factor, "upload_s": t_upload,
                    "levels": int(ex["lev_ptr"].size - 1), "fronts": int(ex["f"].size),
                    "factor_MB": ex["data"].nbytes / 1e6,
                    "psolve_ms": ps_ms,
                    "roofline_psolve": {"bound": "hbm", "achieved": nb / (ps_ms * 1e-3) / 1e9,
                                        "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                        "frac": nb / (ps_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                        "bytes_per_call": int(nb)}})
                # the host loop with the host solve of the same factors
                uh = torch.zeros_like(ft)
                t0 = time.perf_counter()
                _, it_h, _ = pr.precond_solve(ft, uh, F.solve, rtol=1e-8, restart=40, maxit=400)
                entry["host_loop"] = {"iterations": it_h,
                                      "solve_ms": (time.perf_counter() - t0) * 1e3}
                res["graph"] = entry
            else:
                res["direct"] = entry
            pr.close()
        out["cases"][label] = res
    return out


def section_3d_t2(dev, reps):
    """Setup with 5x5x5 stencils (t = 2) on the 3D Helmholtz field, n = 64."""
    import torch
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import workloads as W
    q = W.helm3d_random(64, t=2)
    m = (2 * q.t + 1) ** 3
    pr = lsp.Problem(3, q.n, torch.from_numpy(q.v.reshape(-1)).to(dev))
    Pq = torch.empty(q.N * m, dtype=torch.float64, device=dev)
    iq = torch.empty(q.N, dtype=torch.int32, device=dev)
    fn = lambda: pr.stencil_setup(q.t, q.num_shifts, Pq, iq)
    for _ in range(3):
        fn()
    stream = torch.cuda.current_stream(dev)
    ts = timed(stream, fn, reps)
    pr.profile(True)
    for _ in range(reps):
        fn()
    prof = pr.profile_read()
    pr.profile(False)
    pr.close()
    stage = {k: prof[k][0] / max(prof[k][1], 1) for k in ("shifts", "green", "null", "assemble")}
    nbytes = q.N * (8 + 8 * m + 4)
    return {"workload": f"3D Helmholtz, smooth random c in [0.8,1.2], n={q.n} (N={q.N}), "
                        f"t={q.t} (5x5x5 stencils), |S|={q.num_shifts}",
            "setup_ms": ts * 1e3, "stencils_per_s": q.N / ts, "stage_ms_profiled": stage,
            "assemble_hbm_frac": nbytes / (stage["assemble"] * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-versus-exact setup section")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form section")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the non-localized and 3D t = 2 sections")
    ap.add_argument("--krylov-only", action="store_true",
                    help="only run the device-GMRES section (for profiling its kernels)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="only run 5 device-to-device copies of MiB mebibytes and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the hot path is a single-GPU build); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1607_02560_amd import lsp
    from paper_1607_02560_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe:
        # reference for the FETCH_SIZE / WRITE_SIZE counters: each copy reads
        # and writes exactly copy_probe MiB
        nbytes = args.copy_probe << 20
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 5}))
        return
    if args.krylov_only:
        print(json.dumps({"krylov_device": krylov_section(dev, args.steps)}))
        return
    p = W.helm2d_random(args.n)
    d, n, t, N = p.d, p.n, p.t, p.N
    m = (2 * t + 1) ** d
    print(f"[bench] workload {p.name} n={n} t={t} |S|={p.num_shifts} N={N}", file=sys.stderr,
          flush=True)
    v = torch.from_numpy(p.v.reshape(-1)).to(dev)
    u = torch.from_numpy(p.f.reshape(-1)).to(dev)
    r = np.random.default_rng(1)
    u += torch.from_numpy(r.standard_normal(N) + 1j * r.standard_normal(N)).to(dev)
    y = torch.empty_like(u)
    P = torch.empty(N * m, dtype=torch.float64, device=dev)
    idx = torch.empty(N, dtype=torch.int32, device=dev)
    prob = lsp.Problem(d, n, v)

    def step():
        prob.stencil_setup(t, p.num_shifts, P, idx)
        prob.ps_apply(u, y)

    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the K timed steps (setup + apply), bracketed by device synchronisation
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # setup alone and apply alone, max(K, 100) calls each (after W setups of
    # their own: the step loop above interleaves the apply)
    reps = max(args.steps, 100)
    for _ in range(args.warmup):
        prob.stencil_setup(t, p.num_shifts, P, idx)
    t_setup = timed(stream, lambda: prob.stencil_setup(t, p.num_shifts, P, idx), reps)
    t_apply = timed(stream, lambda: prob.ps_apply(u, y), reps)
    # the C-apply z = C r of the preconditioner (once per GMRES iteration) on
    # the tables of this setup
    zc = torch.empty_like(u)
    for _ in range(args.warmup):
        prob.c_apply(u, zc)
    t_capply = timed(stream, lambda: prob.c_apply(u, zc), reps)
    del zc
    # the FP32-storage form: same FP64 setup, P rows rounded to float32
    P32 = torch.empty(N * m, dtype=torch.float32, device=dev)
    setup32 = lambda: prob.stencil_setup(t, p.num_shifts, P32, idx, precision=lsp.LSP_FP32_REFINE)
    for _ in range(args.warmup):
        setup32()
    t_setup32 = timed(stream, setup32, reps)
    del P32
    # the non-localized setup of Sec. 3 (one shift, the mean of v) on the
    # same field and buffers
    if not args.no_extras:
        setup_g = lambda: prob.stencil_setup_global(t, P, idx)
        for _ in range(args.warmup):
            setup_g()
        t_setup_g = timed(stream, setup_g, reps)
    # per-stage HIP events recorded by the library on its stream (direct
    # launches): the dominant kernel's average duration for the roofline
    prob.profile(True)
    for _ in range(args.steps):
        step()
    prof = prob.profile_read()
    prob.profile(False)
    tab = prob.get_tables()

    def avg_ms(stage):
        tot, cnt = prof[stage]
        return tot / max(cnt, 1)

    nb = algorithmic_bytes(N, m)
    t_asm = avg_ms("assemble") * 1e-3
    asm_gbps = nb["assemble"] / t_asm / 1e9
    apply_gbps = nb["apply"] / t_apply / 1e9
    capply_gbps = nb["c_apply"] / t_capply / 1e9
    out = {
        "metric": METRIC,
        "value": N / t_setup,
        "unit": "stencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Helmholtz, smooth random c in [0.8,1.2], n={n} "
                               f"(N={N}), t={t} (5x5 stencils), |S|={p.num_shifts}",
                   "d": d, "n": n, "t": t, "num_shifts": p.num_shifts,
                   "num_shifts_effective": int(len(tab["S"]))},
        "setup_ms": t_setup * 1e3,
        "setup_hbm_frac": nb["setup"] / t_setup / 1e9 / HBM_PEAK_GBPS,
        "ps_apply_ms": t_apply * 1e3,
        "ps_apply_GBps": apply_gbps,
        "ps_apply_per_s": 1.0 / t_apply,
        "stage_ms_profiled": {k: avg_ms(k) for k in ("shifts", "green", "null", "assemble",
                                                      "setup", "apply")},
        "roofline": {"kernel": "assemble_kernel (per-point P rows)", "bound": "hbm",
                     "achieved": asm_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": asm_gbps / HBM_PEAK_GBPS, "traffic": assemble_traffic(),
                     "bytes_per_launch": nb["assemble"]},
        "form_fp32_refine": {"setup_ms": t_setup32 * 1e3, "stencils_per_s": N / t_setup32,
                             "bytes_per_setup": N * (8 + 4 * m + 4),
                             "hbm_frac": N * (8 + 4 * m + 4) / t_setup32 / 1e9 / HBM_PEAK_GBPS},
        "roofline_ps_apply": {"bound": "hbm", "achieved": apply_gbps, "peak": HBM_PEAK_GBPS,
                              "unit": "GB/s", "frac": apply_gbps / HBM_PEAK_GBPS,
                              "bytes_per_call": nb["apply"]},
        "c_apply_ms": t_capply * 1e3,
        "roofline_c_apply": {"bound": "hbm", "achieved": capply_gbps, "peak": HBM_PEAK_GBPS,
                             "unit": "GB/s", "frac": capply_gbps / HBM_PEAK_GBPS,
                             "bytes_per_call": nb["c_apply"]},
    }
    if not args.no_extras:
        # the launch-shape tuner on the same problem (after the measurements
        # above, which use the built-in shapes)
        out["autotune"] = {"choices_and_ms": prob.autotune(t, p.num_shifts, P, u, y, reps=5),
                           "note": "fastest candidate per shape; the headline uses the "
                                   "built-in shapes"}
        prob.set_tuning()
        out["non_localized"] = non_localized_section(dev, t_setup_g, N)
        # the per-point radius of Sec. 4.2 (leaf box 8, t <= 2) on the same field
        setup_nd = lambda: prob.stencil_setup_nd(8, p.num_shifts, P, idx)
        for _ in range(args.warmup):
            setup_nd()
        t_nd = timed(stream, setup_nd, reps)
        out["form_nd_radius"] = {"leaf": 8, "t_max": 2, "setup_ms": t_nd * 1e3,
                                 "stencils_per_s": N / t_nd}
    prob.close()
    del P, idx
    if not args.no_extras:
        out["form_3d_t2"] = section_3d_t2(dev, args.steps)
        print("[bench] device GMRES with the nested-dissection P-solve", file=sys.stderr,
              flush=True)
        out["krylov_device"] = krylov_section(dev, args.steps)
    if not args.no_learned:
        out["learned_vs_exact"] = learned_vs_exact(dev, stream, args.steps, args.train_steps)
    if not args.no_batched:
        out["form_batched"] = batched_section(dev, args.steps)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
