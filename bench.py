#!/usr/bin/env python
"""Benchmark of the GKSL -> real-ODE hot path on one MI355X.

Workload (default): dense random Lindbladians with N = 200 (M = N^2 - 1 =
39999): 8 ensemble realizations (seeds 0..7), each with a GUE Hamiltonian and
a Wishart Kossakowski matrix gamma = N W W^+ / Tr(W W^+) (W complex Ginibre,
M x M, 25.6 GB in complex128), assembled into Q (12.8 GB, FP64) and K and held
on the device, then 16 pure initial states per realization propagated by
classic RK4 with dt = 1e-3, all 8 x 16 states in one batched launch sequence.

One "step" of this script is one batched RK4 step: 4 stage products over the
8 resident systems (8 x 4 passes over a 12.8 GB Q) advancing 8 x 16 states by
dt. After the inputs are prepared, --warmup untimed steps run, then exactly
--steps timed steps in one call, bracketed by device synchronization (and HIP
events on the library's stream). value = realizations x steps / timed seconds:
RK4 steps per second of one 16-state block. The whole 1000-step job of the
configuration runs with --full-job.

Each realization's assembly (lindblad_prepare with gamma resident in HBM) is
timed once (after one untimed warm-up preparation of realization 0), before the RK4
steps, and reported as assembly_s_per_realization;
gamma is drawn on the device outside that timer (the 8 gamma matrices, 205 GB,
do not fit in HBM next to the 8 resident Q).

The JSON line also carries the roofline of the dominant kernel (the RK4 stage
GEMM over all 8 systems, timed with HIP events on the stream it runs on) and
the CPU oracle timed on a bounded sample of the same workload: RK4 steps of a
16-state block on realization 0's Q, and the assembly of sampled rows of every
class of realization 0 (all diagonal rows), scaled to the whole Q.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q,K assembly s + RK4 steps/s at N=200 dense; batched solves/s, p99 vs plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def gemm64_digest():
    """Digest of the FP64 stage-GEMM source: its work mapping and the direct and
    LDS-staged kernel bodies."""
    src = open(os.path.join(ROOT, "paper_1912_01491_amd", "csrc", "propagate.hip")).read()
    a = src.index("struct GemmGrid")
    b = src.index("template <int RT, int CT, bool ALIGNED>", src.index("void k_gemm64"))
    c = src.index("// LDS-staged variants")
    d = src.index("template <int RT, int CT>", src.index("void k_gemm64s"))
    return hashlib.sha256((src[a:b] + src[c:d]).encode()).hexdigest()[:16]


def staged(Qs, ldq, elem):
    """True when the stage GEMM runs its LDS-staged form (128-byte rows)."""
    return (ldq * elem) % 128 == 0 and all(q.data_ptr() % 128 == 0 for q in Qs)


def measured_traffic(M, R, B, tile):
    """HBM bytes per launch of k_gemm64 from the FETCH_SIZE / WRITE_SIZE counter
    runs summarised under profiles/, scaled by the copy-kernel factors recorded
    there; None unless kernel source, shape and tile are those of the counter run."""
    path = os.path.join(ROOT, "profiles", "k_gemm64s_traffic_N200_dense.md")
    try:
        line = next(x for x in open(path) if x.startswith("traffic-record:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    same_tile = all(rec["tile"][k] == tile[k] for k in ("rows", "kslab", "waves"))
    if (rec["M"], rec["systems"], rec["states"]) != (M, R, B) or not same_tile or rec["source_digest"] != gemm64_digest():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def assembly_traffic(N, M, ldq):
    """Measured HBM bytes of one dense preparation (all assembly kernels) from the
    FETCH_SIZE / WRITE_SIZE runs summarised under profiles/, scaled by the copy
    factors recorded there; None unless the assembly source and the shape are those
    of the counter runs."""
    path = os.path.join(ROOT, "profiles", "k_quad_assembly_N200_dense.md")
    try:
        line = next(x for x in open(path) if x.startswith("traffic-record:"))
    except (OSError, StopIteration):
        return None
    rec = json.loads(line.split(":", 1)[1])
    src = open(os.path.join(ROOT, "paper_1912_01491_amd", "csrc", "prepare_dense.hip")).read()
    digest = hashlib.sha256(src.encode()).hexdigest()[:16]
    if (rec["N"], rec["M"], rec["ldq"]) != (N, M, ldq) or rec["source_digest"] != digest:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps (default config: batched RK4 steps over all realizations and states)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed ones")
    ap.add_argument("--full-job", action="store_true",
                    help="default config: time the configuration's whole job (--rk4-steps batched RK4 steps, "
                         "no warmup) instead of --steps")
    ap.add_argument("--no-check-psd", dest="check_psd", action="store_false",
                    help="default config: skip the Cholesky factorisation of realization 0's gamma (the check that "
                         "it is positive definite to FP64 rounding, untimed)")
    ap.add_argument("--cpu-rows", type=int, default=256,
                    help="default config: sampled S rows (and the J rows of the same pairs) in the oracle's "
                         "assembly sample")
    ap.add_argument("--N", type=int, default=200)
    ap.add_argument("--realizations", type=int, default=8)
    ap.add_argument("--states", type=int, default=16)
    ap.add_argument("--rk4-steps", type=int, default=1000)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--graph", action="store_true", help="replay the RK4 launches from a HIP graph")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle RK4 steps in the CPU sample")
    ap.add_argument("--config", choices=["c1", "c2", "c2p", "c3", "c4", "c5", "c5r", "c6", "c6s", "c7", "c8"],
                    default="c4",
                    help="c4: the N=200 dense headline (default); c1: N=8 dense; c2: N=1000 sparse dimer; "
                         "c3: N=100 dense, 64 states, FP64 vs FP32; c5: serving mix (prepare per request); "
                         "c5r: serving mix on resident systems; c2p: the periodically rocked dimer (one period); "
                         "c6 / c6s: steady states; c7: saved systems; c8: spectrum of Q (Fig. 5)")
    ap.add_argument("--drive-N", type=int, default=1000, help="c2p: Hilbert-space dimension")
    ap.add_argument("--drive-steps", type=int, default=20000, help="c2p: RK4 steps per drive period")
    ap.add_argument("--serving", action="store_true", help="same as --config c5")
    ap.add_argument("--resident", action="store_true", help="with --serving: same as --config c5r")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for rocprofv3 --pmc runs: one plain 4 GiB copy, then the C4 stage GEMM on stand-in Q")
    ap.add_argument("--pmc-c3", action="store_true",
                    help="for rocprofv3 --pmc runs: C3's stage GEMM (N=100, 64 states), 10 launches in FP64 then 10 in "
                         "FP32, default tiles")
    ap.add_argument("--pmc-assembly", action="store_true",
                    help="for rocprofv3 --pmc runs: one plain 4 GiB copy, then one dense preparation at --N")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--arrival", choices=["burst", "poisson"], default="burst")
    ap.add_argument("--ss-N", type=int, default=1000, help="c6s: dimer size")
    ap.add_argument("--spec-N", type=int, default=64, help="c8: Hilbert-space dimension of the spectrum")
    ap.add_argument("--spec-oracle-max-M", type=int, default=10000,
                    help="c8: largest M with the oracle's whole spectrum as baseline and check (above: a scaled "
                         "sample and size-independent checks)")
    ap.add_argument("--persist-dir", default=None, help="c7: directory for the saved files (default: temp dir)")
    ap.add_argument("--ss-maxit", type=int, default=6000, help="c6s: GMRES iteration limit")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="Poisson arrival rate (requests/s); 0 with --arrival poisson: --rate-frac x the plain "
                         "path's throughput measured on a burst of the first --rate-sample requests")
    ap.add_argument("--rate-frac", type=float, default=0.8)
    ap.add_argument("--rate-sample", type=int, default=400)
    ap.add_argument("--fp32-share", type=float, default=0.0,
                    help="c5/c5r: share of dense requests that opt in to FP32 matrix-core integration")
    ap.add_argument("--slots", type=int, default=6)
    ap.add_argument("--max-batch", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=48.0)
    ap.add_argument("--serve-steps", type=int, default=500)
    return ap.parse_args()


def _serving_inputs(args, ctx, lb, wl, torch, np):
    """The serving mix of configuration C5: a device-resident pool of 4 dense
    random Lindbladians per N (gamma drawn on the device for N >= 64), one
    static dimer per N, and `requests` requests (N uniform in {16, 32, 64, 96,
    128}, 70 % dense / 30 % dimer, one pure state each, seed 1000 + i)."""
    dev = torch.device("cuda", 0)
    g = wl.rng(2024)
    Ns = [16, 32, 64, 96, 128]
    pool = {}
    for N in Ns:
        for r in range(4):
            H = torch.from_numpy(wl.gue_hamiltonian(N, 500 + 10 * N + r)).to(dev)
            if N <= 32:
                gamma = torch.from_numpy(wl.wishart_kossakowski(N, 600 + 10 * N + r)).to(dev)
            else:
                gamma = wl.wishart_kossakowski_device(N, 600 + 10 * N + r, device=dev)
            pool[(N, r)] = (H, gamma)
        log("gamma pool for N=%d ready" % N)
    dimers = {}
    for N in Ns:
        H, rates, Ls = wl.dimer_model(N)
        dimers[N] = (tuple(torch.from_numpy(x).to(dev) for x in wl.to_csr(H)), rates,
                     [tuple(torch.from_numpy(x).to(dev) for x in wl.to_csr(L)) for L in Ls])
    reqs = []
    gp = wl.rng(2025)  # FP32 opt-in draws, independent of the request mix
    for i in range(args.requests):
        N = int(g.choice(Ns))
        kind = "dense" if g.random() < 0.7 else "sparse"
        psi = torch.from_numpy(wl.random_pure_state(N, 1000 + i)[None, :]).to(dev)
        V0 = lb.lb_expand_pure(ctx, psi)
        prec = lb.FP32 if (kind == "dense" and gp.random() < args.fp32_share) else lb.FP64
        reqs.append((kind, N, int(g.integers(0, 4)), V0, prec))
    torch.cuda.synchronize()
    log("%d requests ready (%d dense, %d of them FP32)" % (len(reqs), sum(r[0] == "dense" for r in reqs),
                                                          sum(r[4] == lb.FP32 for r in reqs)))
    return Ns, pool, dimers, reqs


def _poisson_arrivals(n, rate):
    """Arrival times (s) of a Poisson stream of `n` requests at `rate` per second (seeded)."""
    from paper_1912_01491_amd import workloads as wl
    import numpy as np
    return np.cumsum(wl.rng(4242).exponential(1.0 / rate, size=n))


def _serve(args, lb, np, reqs, arrivals, slots, max_batch, label, Ns, submit, setup=None):
    """Runs the request list through one server: a feeder thread submits each
    request at its arrival time, the main thread waits in order. Returns wall
    time, latencies (completion - submission, the submission being the
    arrival), stats and outputs."""
    import threading

    srv = lb.Server(0, budget_bytes=int(args.budget_gb * (1 << 30)), slots=slots, max_batch=max_batch,
                    max_N=max(Ns))
    ctxinfo = setup(srv) if setup else None
    tickets = [None] * len(reqs)

    def feeder():
        t0 = time.perf_counter()
        for i, req in enumerate(reqs):
            d = arrivals[i] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets[i] = submit(srv, ctxinfo, req)

    t_start = time.perf_counter()
    th = threading.Thread(target=feeder)
    th.start()
    # wait in submission order while the feeder is still submitting
    for i in range(len(reqs)):
        while tickets[i] is None and th.is_alive():
            time.sleep(0.001)
        if tickets[i] is None:  # the feeder ended early (it raised)
            break
        srv.wait(tickets[i][0])
        if (i + 1) % 100 == 0:
            log("%s: %d of %d requests done after %.1f s" % (label, i + 1, len(reqs), time.perf_counter() - t_start))
    th.join()
    if any(t is None for t in tickets):
        srv.close()
        raise RuntimeError("%s: the feeder stopped before submitting every request" % label)
    wall = time.perf_counter() - t_start
    lat = np.array([srv.times(t)[2] - srv.times(t)[0] for t, _ in tickets])
    st = srv.stats()
    outs = [v for _, v in tickets]
    srv.close()
    log("%s: %d requests in %.2f s (%.2f solves/s), p50 %.3f s, p99 %.3f s, %s"
        % (label, len(reqs), wall, len(reqs) / wall, np.percentile(lat, 50), np.percentile(lat, 99), st))
    return wall, lat, st, outs


def serving(args):
    """Serving mix (configuration C5): N uniform in {16, 32, 64, 96, 128}; 70%
    dense random Lindbladians (gamma from a device-resident pool of 4
    realizations per N), 30% static dimers (sparse path); each request is one
    pure state integrated for `serve-steps` RK4 steps. Two modes:
      * c5 (default): every request carries its Lindbladian and is prepared
        (Q, K) and integrated by the server;
      * c5r (--resident): the 25 distinct Lindbladians of the pool are
        registered once (Q, K resident) and requests only carry states, so the
        server integrates up to 16 requests on the same system per pass over Q.
    The same request list runs through the continuous-batching server and
    through the plain path (one slot, no batching: first-in first-out, one
    request at a time); their results must agree bit for bit."""
    import numpy as np
    import torch

    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    resident = args.config == "c5r" or args.resident
    ctx = lb.Context(0)
    Ns, pool, dimers, reqs = _serving_inputs(args, ctx, lb, wl, torch, np)

    if resident:
        def setup(srv):
            t0 = time.perf_counter()
            sids = {}
            for (N, r), (H, gamma) in pool.items():
                sids[("dense", N, r)] = srv.register_dense(H, gamma)
            for N, (Hc, rates, Lc) in dimers.items():
                sids[("sparse", N, 0)] = srv.register_sparse(N, Hc, rates, Lc)
            log("registered %d systems in %.2f s" % (len(sids), time.perf_counter() - t0))
            return sids

        def submit(srv, sids, req):
            kind, N, r, V0, prec = req
            return srv.submit_system(sids[(kind, N, r if kind == "dense" else 0)], V0, args.dt, args.serve_steps,
                                     precision=prec)
    else:
        setup = None

        def submit(srv, _, req):
            kind, N, r, V0, prec = req
            if kind == "dense":
                H, gamma = pool[(N, r)]
                return srv.submit_dense(H, gamma, V0, args.dt, args.serve_steps, precision=prec)
            Hc, rates, Lc = dimers[N]
            return srv.submit_sparse(N, Hc, rates, Lc, V0, args.dt, args.serve_steps)

    if resident and args.fp32_share > 0:
        raise SystemExit("c5r registers FP64 systems; --fp32-share is for c5")
    mb = max(args.max_batch, 16) if resident else args.max_batch
    rate, rate_from = args.rate, "given"
    if args.arrival == "poisson":
        if rate <= 0:
            sample = reqs[:args.rate_sample]
            w0, _, _, _ = _serve(args, lb, np, sample, np.zeros(len(sample)), 1, 1, "plain (rate sample)", Ns,
                                 submit, setup)
            rate = args.rate_frac * len(sample) / w0
            rate_from = ("%.2f x the plain path's throughput on a burst of the first %d requests (%.3f solves/s)"
                         % (args.rate_frac, len(sample), len(sample) / w0))
        arrivals = _poisson_arrivals(len(reqs), rate)
        log("Poisson arrivals at %.3f requests/s (%s)" % (rate, rate_from))
    else:
        arrivals = np.zeros(len(reqs))
    w_s, lat_s, st_s, out_s = _serve(args, lb, np, reqs, arrivals, args.slots, mb, "served", Ns, submit, setup)
    w_p, lat_p, st_p, out_p = _serve(args, lb, np, reqs, arrivals, 1, 1, "plain", Ns, submit, setup)
    same = all(torch.equal(a, b) for a, b in zip(out_s, out_p))
    fp32 = None
    i32 = [i for i, r in enumerate(reqs) if r[4] == lb.FP32]
    if i32:
        # the FP32 requests again in FP64 (alone, one slot) and, for N <= 32, the oracle
        ref = [(r[0], r[1], r[2], r[3], lb.FP64) for r in (reqs[i] for i in i32)]
        _, _, _, out64 = _serve(args, lb, np, ref, np.zeros(len(ref)), 1, 1, "FP64 reference of the FP32 requests",
                                Ns, submit, setup)
        errs = []
        for i, v64 in zip(i32, out64):
            a, b = out_s[i].cpu().numpy(), v64.cpu().numpy()
            errs.append(float(np.abs(a - b).max() / np.abs(b).max()))
        import oracle
        oracle.build()
        oerrs = []
        for i in i32:
            kind, N, r, V0, _ = reqs[i]
            if N > 32 or len(oerrs) >= 20:
                continue
            H, gamma = pool[(N, r)]
            Qo, Ko = oracle.prepare_dense(H.cpu().numpy(), gamma.cpu().numpy())
            Vo = oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), args.dt, args.serve_steps)
            oerrs.append(float(np.abs(out_s[i].cpu().numpy() - Vo).max() / np.abs(Vo).max()))
        fp32 = {"requests": len(i32), "rel_err_vs_fp64_max": max(errs), "rel_err_vs_fp64_median": float(np.median(errs)),
                "oracle_sample": len(oerrs), "rel_err_vs_oracle_max": max(oerrs) if oerrs else None,
                "note": "normwise relative error of each FP32 request's final state against the same request "
                        "integrated in FP64 by the library, and against the FP64 oracle for FP32 requests with "
                        "N <= 32 (up to 20)"}
        log("FP32 requests: max rel err vs FP64 %.2e (median %.2e), vs oracle %s"
            % (fp32["rel_err_vs_fp64_max"], fp32["rel_err_vs_fp64_median"], fp32["rel_err_vs_oracle_max"]))
    mode = ("resident systems (25 registered Lindbladians, requests carry states only)" if resident
            else "prepare per request")
    out = {
        "metric": "batched solves/s, p99 vs plain (serving mix)",
        "value": len(reqs) / w_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64" if not i32 else "f64 (%.0f%% of dense requests f32)" % (100 * args.fp32_share),
        "data": "synthetic",
        "config": {"workload": "serving mix: %d requests, N uniform in %s, 70%% dense random / 30%% sparse dimer, "
                               "%d RK4 steps dt=%g, one pure state each, %s arrivals, %s"
                               % (len(reqs), Ns, args.serve_steps, args.dt, args.arrival, mode),
                   "slots": args.slots, "max_batch": mb, "budget_gb": args.budget_gb,
                   "rate": rate, "rate_from": rate_from if args.arrival == "poisson" else None,
                   "fp32_share": args.fp32_share, "resident": bool(resident)},
        "latency": "completion - arrival (each request is submitted at its arrival time)",
        "fp32": fp32,
        "served": {"solves_per_s": len(reqs) / w_s, "p50_s": float(np.percentile(lat_s, 50)),
                   "p99_s": float(np.percentile(lat_s, 99)), "wall_s": w_s, "stats": st_s},
        "plain": {"solves_per_s": len(reqs) / w_p, "p50_s": float(np.percentile(lat_p, 50)),
                  "p99_s": float(np.percentile(lat_p, 99)), "wall_s": w_p, "stats": st_p},
        "served_equals_plain_bitwise": bool(same),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(Q0, K0, V0, steps: int, N: int, H0=None, gamma0=None, nrows: int = 64):
    """The oracle (plain C, OpenMP over rows) on a bounded sample of the default
    workload, realization 0:
      * RK4: `steps` RK4 steps of the 16-state block V0 on the host copy Q0 of
        the realization's Q (the same matrix the GPU integrates);
      * assembly (when gamma0 is given): Q rows sampled from every class --
        `nrows` random S rows with the J rows of the same pairs, and all N - 1
        diagonal rows -- and K, timed per class and scaled by the class sizes
        to the whole Q; the oracle's fixed cost (its f/d table and K) is timed once
        with no rows and counted once. The sampled rows and K are compared
        with the GPU's (Q0, K0, host copies): normwise relative error over the
        sample.
    """
    import numpy as np

    import oracle

    oracle.build()
    M = N * N - 1
    B = V0.shape[0]
    oracle.rk4_dense(Q0[:64, :64].copy(), np.zeros(64), V0[:, :64].copy(), 1e-3, 1)  # load / warm the library
    t0 = time.perf_counter()
    oracle.rk4_dense(Q0, np.zeros(M), V0, 1e-3, steps)
    dt = time.perf_counter() - t0
    rate = steps / dt
    out = {"value": rate, "unit": "RK4 steps/s per 16-state block (N=200)", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": "%d RK4 steps of a %d-state block on realization 0's Q (M=%d, the full workload's matrix); "
                     "%.2f s" % (steps, B, M, dt)}
    if gamma0 is None:
        return out
    P = N * (N - 1) // 2
    g = np.random.default_rng(7)
    rs = np.sort(g.choice(P, nrows, replace=False))
    groups = {"pair": np.concatenate([rs, P + rs]), "D": np.arange(2 * P, M)}
    sizes = {"pair": 2 * P, "D": N - 1}
    log("cpu baseline: oracle assembly sample (%d S, %d J, %d D rows) at N=%d" % (nrows, nrows, N - 1, N))
    t = time.perf_counter()
    _, K_or = oracle.prepare_dense(H0, gamma0, rows=np.arange(0))
    t_fixed = time.perf_counter() - t
    est = t_fixed
    per = {}
    err_q = 0.0
    qref = 0.0
    for cls, rows in groups.items():
        t = time.perf_counter()
        Qr, _ = oracle.prepare_dense(H0, gamma0, rows=rows)
        tc = time.perf_counter() - t
        per[cls] = tc
        est += max(tc - t_fixed, 0.0) * sizes[cls] / len(rows)
        err_q = max(err_q, float(np.abs(Q0[rows] - Qr).max()))
        qref = max(qref, float(np.abs(Qr).max()))
        log("cpu baseline: %s rows %.2f s (fixed part %.2f s)" % (cls, tc, t_fixed))
    err_k = float(np.abs(K0 - K_or).max() / np.abs(K_or).max())
    out["assembly_s_per_realization"] = est
    out["assembly_sample"] = (
        "oracle rows of realization 0: %d random S rows with the %d J rows of the same pairs (%.2f s), all %d "
        "diagonal rows (%.2f s), each call including the oracle's fixed part (its f/d table and K, %.2f s alone); "
        "whole Q estimated as fixed + sum over the two classes of (call - fixed) x class size / rows sampled"
        % (nrows, nrows, per["pair"], N - 1, per["D"], t_fixed))
    out["assembly_parity"] = {"rows": int(sum(len(r) for r in groups.values())),
                              "rel_err_Q_rows": err_q / qref, "rel_err_K": err_k}
    return out


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def config_c1(args):
    """N=8 (M=63) dense random Lindbladian, H = (G+G^+)/2, Wishart gamma; one
    random pure state (and a 16-state block), 1000 RK4 steps dt=1e-3. Latency
    bound: Q (31.8 KB) stays in one workgroup's LDS for the whole run."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, S, dt = 8, 1000, 1e-3
    H, gamma = wl.random_lindbladian(N, 0, hamiltonian="plain")
    ctx = lb.Context(0)
    Hd, Gd = torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda()
    res = {}
    for B in (1, 16):
        psis = torch.from_numpy(wl.random_pure_states(N, B, 1)).cuda()
        lb.lindblad_prepare(ctx, Hd, Gd)
        t_prep = min(_timed(lambda: lb.lindblad_prepare(ctx, Hd, Gd))[0] for _ in range(20))
        Q, K = lb.lindblad_prepare(ctx, Hd, Gd)
        V0 = lb.lb_expand_pure(ctx, psis)
        V = V0.clone()
        lb.lindblad_propagate(ctx, Q, K, V, dt, S)
        ts = []
        for _ in range(5):
            V = V0.clone()
            ts.append(_timed(lambda: lb.lindblad_propagate(ctx, Q, K, V, dt, S))[0])
        t_prop = min(ts)
        Qo, Ko = oracle.prepare_dense(H, gamma)
        Vo = oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), dt, S)
        err = float(np.abs(V.cpu().numpy() - Vo).max() / np.abs(Vo).max())
        t0 = time.perf_counter()
        oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), dt, S)
        t_cpu = time.perf_counter() - t0
        res[B] = {"assembly_us": 1e6 * t_prep, "rk4_steps_per_s": S / t_prop, "run_ms": 1e3 * t_prop,
                  "rel_err_vs_oracle": err, "oracle_rk4_steps_per_s": S / t_cpu}
        log("C1 B=%d: assembly %.1f us, %.0f RK4 steps/s, err %.1e" % (B, 1e6 * t_prep, S / t_prop, err))
    out = {"metric": "C1: N=8 dense assembly us and RK4 steps/s", "value": res[1]["rk4_steps_per_s"],
           "unit": "RK4 steps/s (1 state, N=8)", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "dense random Lindbladian N=8 (M=63), H=(G+G^+)/2, Wishart gamma, "
                                  "1000 RK4 steps dt=1e-3", "states": [1, 16]},
           "results": {str(k): v for k, v in res.items()},
           "cpu_baseline": {"value": res[1]["oracle_rk4_steps_per_s"], "unit": "RK4 steps/s (1 state, N=8)",
                            "cores": oracle.num_threads(), "kind": "oracle", "sample": "the whole 1000-step run"}}
    ctx.close()
    print(json.dumps(out), flush=True)


def config_c2(args):
    """Bosonic dimer, N=1000 (M=999999), J=1, U=0.5, static, one jump b1^+ b2
    at rate 0.1/(N-1): sparse preparation (CSR) and 1000 RK4 steps dt=1e-3
    of one random pure state."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, S, dt = 1000, 1000, 1e-3
    M = N * N - 1
    H, rates, Ls = wl.dimer_model(N)
    ctx = lb.Context(0)
    Hc = tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(H))
    Lc = [tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(L)) for L in Ls]
    lb.lindblad_prepare_sparse(ctx, N, Hc, rates, Lc)
    t_prep, (rp, col, val, K) = min((_timed(lambda: lb.lindblad_prepare_sparse(ctx, N, Hc, rates, Lc))
                                     for _ in range(3)), key=lambda x: x[0])
    nnz = int(col.numel())
    psi = torch.from_numpy(wl.random_pure_state(N, 0)[None, :]).cuda()
    V0 = lb.lb_expand_pure(ctx, psi)
    V = V0.clone()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, dt, 10)
    V = V0.clone()
    t_prop, _ = _timed(lambda: lb.lindblad_propagate_csr(ctx, rp, col, val, K, V, dt, S))
    # algorithmic bytes per RK4 step: four passes over the stored entries (8 B value + 4 B column index,
    # the kernel's format; its slice padding is not counted) and the CSR row pointers, plus the M-vectors
    # touched once each: per step x in (4),
    # K (4), v read (4) and written (1), accumulator read (3) and written (3), stage output (4)
    bytes_step = 4 * (nnz * (8 + 4) + (M + 1) * 8) + 23 * M * 8
    gbs = S * bytes_step / t_prop / 1e9
    rho = lb.lb_reconstruct(ctx, V, N)[0].cpu().numpy()
    tr = abs(np.trace(rho) - 1)
    # positivity of rho(T): classic RK4 at this dt (spectral radius x dt ~ 2) is not positivity
    # preserving; the smallest eigenvalue is reported, with one run at half the step for comparison
    mineig = float(np.linalg.eigvalsh(0.5 * (rho + rho.conj().T)).min())
    Vh = V0.clone()
    lb.lindblad_propagate_csr(ctx, rp, col, val, K, Vh, 0.5 * dt, 2 * S)
    rho_h = lb.lb_reconstruct(ctx, Vh, N)[0].cpu().numpy()
    mineig_half = float(np.linalg.eigvalsh(0.5 * (rho_h + rho_h.conj().T)).min())
    # oracle parity on sampled rows
    rows = np.array([0, 1, 777, 499499, 499500, 998999, 999000, M - 1])
    Qo, Ko = oracle.prepare_factored(H, rates, Ls, rows)
    rpc, colc, valc = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    Qg = np.zeros((len(rows), M))
    for t, r in enumerate(rows):
        Qg[t, colc[rpc[r]:rpc[r + 1]]] = valc[rpc[r]:rpc[r + 1]]
    err = float(np.abs(Qg - Qo).max() / np.abs(Qo).max())
    log("C2: prepare %.1f ms (nnz %d = %.2f N^2), %d RK4 steps in %.3f s (%.1f us/step, %.0f GB/s)"
        % (1e3 * t_prep, nnz, nnz / N**2, S, t_prop, 1e6 * t_prop / S, gbs))
    out = {"metric": "C2: N=1000 sparse dimer prepare s and RK4 steps/s", "value": S / t_prop,
           "unit": "RK4 steps/s (1 state, N=1000)", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "bosonic dimer N=1000 (M=999999), J=1, U=0.5, eps=0, L=b1^+ b2 at rate "
                                  "0.1/999, 1000 RK4 steps dt=1e-3"},
           "prepare_s": t_prep, "nnz": nnz, "us_per_step": 1e6 * t_prop / S,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sell_stage<false, 1>",
                        "bytes_per_step": bytes_step},
           "checks": {"trace_err": float(tr), "sampled_rows_rel_err_vs_oracle": err,
                      "min_eig_rho_T": mineig, "min_eig_rho_T_half_dt": mineig_half}}
    ctx.close()
    print(json.dumps(out), flush=True)


def config_c2p(args):
    """The periodically rocked dimer of the paper's sparse model (Sec. 3): H(t)
    = H0 + eps(t)(n2 - n1), J = -1, U = 2.2, eps(t) = E + A Theta(t) with
    E = -1, A = -1.5, T = 2 pi; one jump (b1^+ + b2^+)(b1 - b2) at rate
    0.1/(N-1); one period of 20000 RK4 steps from a random pure state. Q0 (H0
    and the dissipator) and Q1 (n2 - n1) are prepared on the device in CSR."""
    import math

    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N = args.drive_N
    M = N * N - 1
    E, A, T = -1.0, -1.5, 2 * math.pi
    S = args.drive_steps
    dt = T / S
    H0, H1, rates, Ls = wl.rocked_dimer_model(N)
    ctx = lb.Context(0)

    def dev_csr(X):
        return tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(X))

    H0c, H1c, Lc = dev_csr(H0), dev_csr(H1), [dev_csr(L) for L in Ls]

    def prep():
        rp0, c0, v0, K = lb.lindblad_prepare_sparse(ctx, N, H0c, rates, Lc)
        rp1, c1, v1, _ = lb.lindblad_prepare_sparse(ctx, N, H1c, [], [])
        return (rp0, c0, v0), (rp1, c1, v1), K

    prep()
    t_prep, (Q0, Q1, K) = min((_timed(prep) for _ in range(3)), key=lambda x: x[0])
    nnz0, nnz1 = int(Q0[1].numel()), int(Q1[1].numel())
    psi = torch.from_numpy(wl.random_pure_state(N, 0)[None, :]).cuda()
    V0 = lb.lb_expand_pure(ctx, psi)
    V = V0.clone()
    lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, V, dt, 20, 0.0, E, A, T)
    V = V0.clone()
    t_prop, _ = _timed(lambda: lb.lindblad_propagate_csr_drive(ctx, Q0, Q1, K, V, dt, S, 0.0, E, A, T))
    # algorithmic bytes per RK4 step: four passes over both matrices (8 B value + 4 B column per stored
    # entry, row pointers) and the M-vectors touched once each (as for the static sparse path)
    bytes_step = 4 * ((nnz0 + nnz1) * (8 + 4) + 2 * (M + 1) * 8) + 23 * M * 8
    gbs = S * bytes_step / t_prop / 1e9
    rho = lb.lb_reconstruct(ctx, V, N)[0].cpu().numpy()
    # oracle parity on sampled rows of both matrices
    P = N * (N - 1) // 2
    rows = np.array([0, 1, N - 2, P - 1, P, 2 * P - 1, 2 * P, M - 1])
    Q0o, Ko = oracle.prepare_factored(H0, rates, Ls, rows)
    Q1o, _ = oracle.prepare_factored(H1, [0.0], [np.zeros((N, N))], rows)

    def rows_dense(Q):
        rp, c, v = (x.cpu().numpy() for x in Q)
        out = np.zeros((len(rows), M))
        for t, r in enumerate(rows):
            out[t, c[rp[r]:rp[r + 1]]] = v[rp[r]:rp[r + 1]]
        return out

    err0 = float(np.abs(rows_dense(Q0) - Q0o).max() / np.abs(Q0o).max())
    err1 = float(np.abs(rows_dense(Q1) - Q1o).max() / np.abs(Q1o).max())
    log("C2p: N=%d prepare %.1f ms (nnz %d + %d), one period of %d RK4 steps in %.3f s (%.1f us/step, %.0f GB/s)"
        % (N, 1e3 * t_prep, nnz0, nnz1, S, t_prop, 1e6 * t_prop / S, gbs))
    out = {"metric": "rocked dimer: RK4 steps/s over one drive period", "value": S / t_prop,
           "unit": "RK4 steps/s (1 state, N=%d)" % N, "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "periodically rocked dimer N=%d (M=%d), J=-1, U=2.2, E=-1, A=-1.5, T=2pi, "
                                  "L=(b1^+ + b2^+)(b1 - b2) at rate 0.1/%d, %d RK4 steps per period"
                                  % (N, M, N - 1, S)},
           "prepare_s": t_prep, "nnz_Q0": nnz0, "nnz_Q1": nnz1, "us_per_step": 1e6 * t_prop / S,
           "period_s": t_prop,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sell_stage<true, 1>",
                        "bytes_per_step": bytes_step},
           "checks": {"trace_err": float(abs(np.trace(rho) - 1)),
                      "herm_err": float(np.abs(rho - rho.conj().T).max()),
                      "sampled_rows_rel_err_vs_oracle": {"Q0": err0, "Q1": err1}}}
    ctx.close()
    print(json.dumps(out), flush=True)


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:
        return os.cpu_count() or 1


def config_c6(args):
    """Steady state of the N=100 random Lindbladian (M=9999): GUE H, Wishart
    gamma drawn on the device, Q and K prepared on the device, then Q v = -K by
    FP64 GMRES without preconditioner (the random model's spectrum keeps away
    from zero). Each GMRES iteration streams Q once, so the solve is bound by
    HBM like the one-state RK4 stage."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, tol = 100, 1e-13
    M = N * N - 1
    ctx = lb.Context(0)
    H = torch.from_numpy(wl.gue_hamiltonian(N, 0)).cuda()
    gamma = wl.wishart_kossakowski_device(N, 1)
    Q, K = lb.lindblad_prepare(ctx, H, gamma)
    del gamma
    torch.cuda.empty_cache()
    lb.lindblad_steady_state(ctx, Q, K, tol=tol)
    t, (v, info) = min((_timed(lambda: lb.lindblad_steady_state(ctx, Q, K, tol=tol)) for _ in range(3)),
                       key=lambda x: x[0])
    # operator applications: one residual per cycle start, one per iteration, one final residual
    apps = info["iterations"] + info["restarts"] + 2
    bytes_q = M * Q.stride(0) * 8
    gbs = apps * bytes_q / t / 1e9
    res = float(((Q[:, :M] @ v + K).norm() / K.norm()).item())
    rho = oracle.reconstruct(N, v.cpu().numpy())
    log("C6: N=%d steady state in %.2f ms, %d iterations (%d restarts), residual %.1e, %.0f GB/s over Q"
        % (N, 1e3 * t, info["iterations"], info["restarts"], res, gbs))
    # the oracle's dense solve of the same system on the host cores
    Qh, Kh = Q[:, :M].cpu().numpy(), K.cpu().numpy()
    oracle.steady_state(Qh[:8, :8] + np.eye(8), Kh[:8])
    t0 = time.perf_counter()
    vo = oracle.steady_state(Qh, Kh)
    tc = time.perf_counter() - t0
    err = float(np.abs(v.cpu().numpy() - vo).max() / np.abs(vo).max())
    out = {"metric": "steady state: N=100 random Lindbladian, Q v = -K (FP64)", "value": 1.0 / t,
           "unit": "solves/s (M=9999)", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "random Lindbladian N=100 (M=9999): GUE H seed 0, Wishart gamma seed 1 (Tr = N); "
                                  "GMRES to ||Qv + K|| <= 1e-13 ||K||, no preconditioner"},
           "solve_s": t, "iterations": info["iterations"], "restarts": info["restarts"],
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "k_mv_dense",
                        "bytes_per_application": bytes_q, "applications": apps},
           "cpu_baseline": {"value": 1.0 / tc, "unit": "solves/s (M=9999)", "cores": _blas_threads(),
                            "kind": "oracle", "sample": "the whole solve: dense LU (LAPACK via numpy) of the same "
                                                        "M=9999 system; %.2f s" % tc},
           "checks": {"residual": res, "rel_err_vs_oracle": err, "trace_err": float(abs(np.trace(rho) - 1)),
                      "min_eig_rho": float(np.linalg.eigvalsh(rho).min())}}
    ctx.close()
    print(json.dumps(out), flush=True)


def _nearest(a, b, chunk=512):
    """Largest distance from a value of a to its nearest value in b."""
    import numpy as np
    worst = 0.0
    for i in range(0, len(a), chunk):
        worst = max(worst, float(np.abs(a[i:i + chunk, None] - b[None, :]).min(axis=1).max()))
    return worst


def config_c8(args):
    """Spectrum of one random Lindbladian (Fig. 5, at the sizes the unblocked QR stage
    reaches): GUE H seed 0, Wishart gamma seed 1, Q prepared on the device,
    all M eigenvalues of Q on the device (Householder reduction to Hessenberg form,
    then the multishift QR iteration: blocks above 256 rows swept by chains of bulges
    chased in LDS windows with matrix-core updates of the rest, one workgroup below),
    and their counts on a
    100 x 100 grid over the spectrum's bounding box, divided by the cell area as in
    Fig. 5."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N = args.spec_N
    M = N * N - 1
    ctx = lb.Context(0)
    H = torch.from_numpy(wl.gue_hamiltonian(N, 0)).cuda()
    gamma = wl.wishart_kossakowski_device(N, 1)
    Q, K = lb.lindblad_prepare(ctx, H, gamma)
    del gamma
    torch.cuda.empty_cache()
    Qv = Q[:, :M]
    full = M <= args.spec_oracle_max_M  # the oracle's whole spectrum and a separate reduction timing
    marks = {}
    t_start = [0.0]

    def progress(stage, frac):
        now = time.perf_counter()
        marks.setdefault(stage, now)
        log("C8: %s %.0f %% at %.1f s" % (stage, 100 * frac, now - t_start[0]))

    if full:
        A = Qv.contiguous()
        t_hess, _ = _timed(lambda: lb.lb_hessenberg(ctx, A))
        del A
        log("C8: N=%d M=%d Hessenberg reduction %.3f s" % (N, M, t_hess))
    else:
        ctx.set_progress(progress)
    torch.cuda.synchronize()
    t_start[0] = time.perf_counter()
    t, (lam, info) = _timed(lambda: lb.lindblad_spectrum(ctx, Qv))
    ctx.set_progress(None)
    if not full:  # the reduction ends where the QR stage's first report comes
        t_hess = marks.get("qr", t_start[0] + t) - t_start[0]
    t_qr = t - t_hess
    log("C8: spectrum in %.3f s (QR stage ~%.3f s): %d sweeps, %d chain steps, %d updates, %d windowed rounds, "
        "%.3g product flops" % (t, t_qr, info["sweeps"], info["chain_steps"], info["updates"], info["rounds"],
                                info["product_flops"]))
    z = lam.cpu().numpy()
    pad = 0.01
    re0, re1 = z.real.min(), z.real.max()
    im0, im1 = z.imag.min(), z.imag.max()
    re0, re1 = re0 - pad * (re1 - re0), re1 + pad * (re1 - re0)
    im0, im1 = im0 - pad * (im1 - im0), im1 + pad * (im1 - im0)
    nx = ny = 100
    t_hist, counts = _timed(lambda: lb.lindblad_spectrum_histogram(ctx, lam, re0, re1, im0, im1, nx, ny))
    density = counts.cpu().numpy() / (((re1 - re0) / nx) * ((im1 - im0) / ny))
    # the QR stage: chains of bulges chased in LDS windows (one workgroup per chain), the rest
    # of each block updated by the window products on the matrix cores; their flops over the
    # stage's wall time (chase and one-workgroup solves included) bound the products' rate
    # from below. A direct sweep would read and write three entries (48 B) per update.
    prod_tfs = info["product_flops"] / t_qr / 1e12
    hess_flops = 10.0 / 3.0 * float(M) ** 3
    fro = float(torch.linalg.norm(Qv).item())
    trace = float(torch.diagonal(Qv).sum().item())
    checks = {"trace_err": float(abs(z.sum() - trace)), "max_real": float(z.real.max()),
              "conjugate_pairs": bool(np.sum(z.imag > 0) == np.sum(z.imag < 0)),
              "sum_abs2_over_normF2": float(np.sum(np.abs(z) ** 2) / fro ** 2),  # <= 1 (Schur)
              "counted": int(counts.sum().item()), "density_max": float(density.max()),
              "cells_occupied": int((counts > 0).sum().item())}
    if full:  # the oracle (LAPACK through numpy) on the same matrix, on the host cores
        Qh = Qv.cpu().numpy()
        oracle.spectrum(Qh[:16, :16])
        t0 = time.perf_counter()
        w = oracle.spectrum(Qh)
        tc = time.perf_counter() - t0
        near = max(_nearest(z, w), _nearest(w, z))
        checks["nearest_dist_max"] = near
        checks["nearest_dist_over_eps_M_normF"] = near / (np.finfo(float).eps * M * fro)
        log("C8: oracle %.2f s; largest nearest-value distance %.2e (||Q||_F %.1f)" % (tc, near, fro))
        base = {"value": 1.0 / tc, "unit": "spectra/s (M=%d)" % M, "cores": _blas_threads(), "kind": "oracle",
                "sample": "the whole spectrum of the same Q (LAPACK dgeev through numpy, eigenvalues only); %.2f s"
                          % tc}
    else:  # bounded sample: the oracle on a 4095 x 4095 stand-in, scaled by M^3
        Ms = 4095
        S = wl.rng(7).standard_normal((Ms, Ms))
        oracle.spectrum(S[:16, :16])
        t0 = time.perf_counter()
        oracle.spectrum(S)
        tc = time.perf_counter() - t0
        est = tc * (M / Ms) ** 3
        log("C8: oracle sample %.2f s at M=%d -> %.0f s estimated at M=%d" % (tc, Ms, est, M))
        base = {"value": 1.0 / est, "unit": "spectra/s (M=%d)" % M, "cores": _blas_threads(), "kind": "oracle",
                "sample": "the oracle's LAPACK call on a seeded %d x %d stand-in (%.2f s), scaled by M^3 to "
                          "%.0f s" % (Ms, Ms, tc, est)}
    log("C8: checks %s" % json.dumps(checks))
    out = {"metric": "spectrum of Q: N=%d random Lindbladian, all M eigenvalues (FP64) and their 100 x 100 grid" % N,
           "value": 1.0 / t, "unit": "spectra/s (M=%d)" % M, "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "random Lindbladian N=%d (M=%d): GUE H seed 0, Wishart gamma seed 1 (Tr = N); "
                                  "eigenvalues of Q, counts on a 100 x 100 grid over their bounding box" % (N, M)},
           "spectrum_s": t, "hessenberg_s": t_hess, "qr_s": t_qr, "histogram_s": t_hist,
           "sweeps": info["sweeps"], "chain_steps": info["chain_steps"], "updates": info["updates"],
           "rounds": info["rounds"], "product_flops": info["product_flops"],
           "roofline": {"bound": "mfma", "achieved": prod_tfs, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                        "frac": prod_tfs / FP64_PEAK_TFS, "traffic": None, "kernel": "k_win_rows + k_win_cols",
                        "flops": info["product_flops"], "rounds": info["rounds"],
                        "note": "flops of the window products (dense 2 w^2 per row or column; the kernels skip the "
                                "30 % of the window factor's 16 x 4 blocks that are zero by its band structure) "
                                "over the QR stage's wall time, which also holds the windowed chase and the "
                                "one-workgroup solves; a direct sweep would move 48 B per update (updates x 48 B)"},
           "hessenberg": {"flops": hess_flops, "tflops": hess_flops / t_hess / 1e12},
           "cpu_baseline": base,
           "checks": checks}
    ctx.close()
    print(json.dumps(out), flush=True)


def config_c6s(args):
    """Steady state of the static dimer (the sparse model of the configurations,
    N=1000, M=999999) with the secular preconditioner: Q in CSR prepared on the
    device, the preconditioner built on the device from H and the jump
    operator (Jacobi eigenbasis of H, bordered rate matrix), then FP64 GMRES."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, tol = args.ss_N, 1e-12
    M = N * N - 1
    ctx = lb.Context(0)
    H, rates, Ls = wl.dimer_model(N)

    def dev_csr(X):
        return tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(X))

    Hc, Lc = dev_csr(H), [dev_csr(L) for L in Ls]
    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, Hc, rates, Lc)
    t_pre, pre = _timed(lambda: lb.Secular(ctx, N, Hc, rates, Lc))
    log("C6s: N=%d preconditioner set up in %.2f s" % (N, t_pre))
    t, (v, info) = _timed(lambda: lb.lindblad_steady_state_csr(ctx, rp, col, val, K, tol=tol, maxit=args.ss_maxit,
                                                               pre=pre))
    log("C6s: solved in %.2f s, %d iterations, residual %.1e" % (t, info["iterations"], info["residual"]))
    Qs = torch.sparse_csr_tensor(rp.cpu(), col.cpu(), val.cpu(), size=(M, M))
    res = float(((Qs @ v.cpu()) + K.cpu()).norm() / K.cpu().norm())
    rho = oracle.reconstruct(N, v.cpu().numpy())
    n1 = float(np.real(np.sum(np.arange(N) * np.diag(rho))))
    # the oracle's dense solve on a bounded sample: the same model at N=60
    Ns = 60
    Hs_, rs_, Ls_ = wl.dimer_model(Ns)
    Qo, Ko = oracle.prepare_factored(Hs_, rs_, Ls_, np.arange(Ns * Ns - 1))
    t0 = time.perf_counter()
    oracle.steady_state(Qo, Ko)
    tc = time.perf_counter() - t0
    out = {"metric": "steady state: N=%d dimer, Q v = -K (FP64, preconditioned GMRES)" % N, "value": 1.0 / (t + t_pre),
           "unit": "solves/s incl. preconditioner set-up (M=%d)" % M, "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "bosonic dimer N=%d (M=%d), J=1, U=0.5, L=b1^+ b2 at rate 0.1/%d; GMRES to "
                                  "||Qv + K|| <= 1e-12 ||K||, secular preconditioner" % (N, M, N - 1)},
           "setup_s": t_pre, "solve_s": t, "iterations": info["iterations"], "restarts": info["restarts"],
           "cpu_baseline": {"value": 1.0 / tc, "unit": "solves/s (M=%d)" % (Ns * Ns - 1), "cores": _blas_threads(),
                            "kind": "oracle",
                            "sample": "dense LU of the same model at N=%d (M=%d), %.2f s; a dense N=%d system "
                                      "(%.0f TB) is beyond the oracle" % (Ns, Ns * Ns - 1, tc, N, 8e-12 * M * M)},
           "checks": {"residual": res, "trace_err": float(abs(np.trace(rho) - 1)),
                      "herm_err": float(np.abs(rho - rho.conj().T).max()),
                      "min_eig_rho": float(np.linalg.eigvalsh(rho).min()), "mean_n1": n1}}
    pre.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def config_c7(args):
    """Saving and loading prepared systems (the paper integrates from stored,
    prepared data, Sec. 5): the N=100 dense random Lindbladian (Q 800 MB) and
    the N=1000 sparse dimer (7.49 M stored entries) written to a file and read
    back, the payload hash recomputed on load. The file system is the box's;
    a file just written may still be in the page cache, so the load rate is
    that of a warm read."""
    import tempfile

    import torch

    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    ctx = lb.Context(0)
    d = args.persist_dir or tempfile.gettempdir()
    out = {}
    N = 100
    H = torch.from_numpy(wl.gue_hamiltonian(N, 0)).cuda()
    gamma = wl.wishart_kossakowski_device(N, 1)
    Q, K = lb.lindblad_prepare(ctx, H, gamma)
    del gamma
    torch.cuda.empty_cache()
    path = os.path.join(d, "lb_c7_dense_%d.bin" % os.getpid())
    t_save, _ = _timed(lambda: lb.save_system(ctx, path, N, K, Q=Q))
    size = os.path.getsize(path)
    t_load, (Q2, K2) = _timed(lambda: lb.load_system(ctx, path))
    M = N * N - 1
    same = bool(torch.equal(Q2[:, :M], Q[:, :M]) and torch.equal(K2, K))
    os.remove(path)
    log("C7: dense N=%d, %.0f MB: save %.3f s (%.2f GB/s), load %.3f s (%.2f GB/s), identical %s"
        % (N, size / 1e6, t_save, size / t_save / 1e9, t_load, size / t_load / 1e9, same))
    out["dense_n100"] = {"bytes": size, "save_s": t_save, "load_s": t_load, "identical": same}
    del Q, Q2
    torch.cuda.empty_cache()
    N = 1000
    Hs, rates, Ls = wl.dimer_model(N)

    def dev_csr(X):
        return tuple(torch.from_numpy(x).cuda() for x in wl.to_csr(X))

    rp, col, val, K = lb.lindblad_prepare_sparse(ctx, N, dev_csr(Hs), rates, [dev_csr(L) for L in Ls])
    path = os.path.join(d, "lb_c7_csr_%d.bin" % os.getpid())
    t_save, _ = _timed(lambda: lb.save_system(ctx, path, N, K, csr=(rp, col, val)))
    size2 = os.path.getsize(path)
    t_load, ((rp2, col2, val2), K2) = _timed(lambda: lb.load_system(ctx, path))
    same2 = bool(torch.equal(col2, col) and torch.equal(val2, val) and torch.equal(K2, K) and torch.equal(rp2, rp))
    os.remove(path)
    log("C7: sparse dimer N=%d, %.0f MB: save %.3f s (%.2f GB/s), load %.3f s (%.2f GB/s), identical %s"
        % (N, size2 / 1e6, t_save, size2 / t_save / 1e9, t_load, size2 / t_load / 1e9, same2))
    out["dimer_n1000"] = {"bytes": size2, "save_s": t_save, "load_s": t_load, "identical": same2}
    res = {"metric": "saved systems: load rate of a prepared N=100 dense system", "value": size / out["dense_n100"]["load_s"] / 1e9,
           "unit": "GB/s (file -> HBM, hash checked)", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "save and load of the prepared N=100 dense random "
                                                       "Lindbladian (Q, K) and the N=1000 sparse dimer (CSR, K)"},
           "results": out}
    ctx.close()
    print(json.dumps(res), flush=True)


def config_c3(args):
    """N=100 (M=9999) dense random Lindbladian, GUE H, Wishart gamma; 64 random
    pure states, 2000 RK4 steps dt=1e-3, FP64 (matrix cores) and FP32 matrix
    core path; the FP32 error is stated per state against the FP64 result, and
    both against the FP64 oracle over the first 20 steps."""
    import numpy as np
    import torch

    import oracle
    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, B, S, dt = 100, 64, 2000, 1e-3
    M = N * N - 1
    H, gamma = wl.random_lindbladian(N, 0)
    ctx = lb.Context(0)
    Hd, Gd = torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda()
    lb.lindblad_prepare(ctx, Hd, Gd)
    t_prep, (Q, K) = min((_timed(lambda: lb.lindblad_prepare(ctx, Hd, Gd)) for _ in range(3)), key=lambda x: x[0])
    Q32 = lb.lindblad_q_to_f32(ctx, Q)
    psis = torch.from_numpy(wl.random_pure_states(N, B, 0)).cuda()
    V0 = lb.lb_expand_pure(ctx, psis)
    res = {}
    for name, prec in (("fp64", lb.FP64), ("fp32", lb.FP32)):
        V = V0.clone()
        lb.lindblad_propagate(ctx, Q, K, V, dt, 2, precision=prec, Q32=Q32)
        V = V0.clone()
        t, _ = _timed(lambda: lb.lindblad_propagate(ctx, Q, K, V, dt, S, precision=prec, Q32=Q32))
        flops = 4 * S * 2.0 * M * M * B
        res[name] = {"seconds": t, "rk4_steps_per_s": S / t, "tflops": flops / t / 1e12, "V": V}
        log("C3 %s: %d steps in %.2f s (%.1f TFLOP/s)" % (name, S, t, flops / t / 1e12))
    V64, V32 = res["fp64"].pop("V"), res["fp32"].pop("V")
    per_state = ((V32 - V64).abs().amax(dim=1) / V64.abs().amax(dim=1)).cpu().numpy()
    # oracle parity over 20 steps (full oracle assembly at N=100)
    Qo, Ko = oracle.prepare_dense(H, gamma)
    Vo = oracle.rk4_dense(Qo, Ko, V0.cpu().numpy(), dt, 20)
    errs = {}
    for name, prec in (("fp64", lb.FP64), ("fp32", lb.FP32)):
        V = V0.clone()
        lb.lindblad_propagate(ctx, Q, K, V, dt, 20, precision=prec, Q32=Q32)
        errs[name] = float(np.abs(V.cpu().numpy() - Vo).max() / np.abs(Vo).max())
    qerr = float(np.abs(Q.cpu().numpy()[:, :M] - Qo).max() / np.abs(Qo).max())
    peak64, peak32 = 78.6, 157.3
    out = {"metric": "C3: N=100 dense, 64 states x 2000 RK4 steps, FP64 vs FP32-MFMA", "value": res["fp64"]["rk4_steps_per_s"],
           "unit": "RK4 steps/s (64-state block, N=100, FP64)", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "dense random Lindbladian N=100 (M=9999), GUE H, Wishart gamma, 64 pure states, "
                                  "2000 RK4 steps dt=1e-3"},
           "assembly_s": t_prep, "assembly_rel_err_vs_oracle": qerr,
           "fp64": dict(res["fp64"], roofline={"bound": "mfma", "achieved": res["fp64"]["tflops"], "peak": peak64,
                                                "unit": "TFLOP/s", "frac": res["fp64"]["tflops"] / peak64}),
           "fp32": dict(res["fp32"], roofline={"bound": "mfma", "achieved": res["fp32"]["tflops"], "peak": peak32,
                                                "unit": "TFLOP/s", "frac": res["fp32"]["tflops"] / peak32}),
           "fp32_rel_err_vs_fp64_per_state_at_T": {"max": float(per_state.max()), "median": float(np.median(per_state)),
                                                    "all": [float(x) for x in per_state]},
           "rel_err_vs_oracle_20_steps": errs}
    ctx.close()
    print(json.dumps(out), flush=True)


def pmc_probe(args):
    """Kernels for the HBM traffic counters: a plain copy of 4 GiB (reads and
    writes 4 GiB: the scale for FETCH_SIZE / WRITE_SIZE), then the stage GEMM at
    the C4 shape (8 systems, M = 39999, 16 states) on stand-in Q matrices
    (traffic does not depend on the values)."""
    import torch

    import paper_1912_01491_amd as lb

    n = 1 << 29  # doubles: 4 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    N, R, B = args.N, args.realizations, args.states
    M = N * N - 1
    ldq = lb.default_ldq(M)
    ctx = lb.Context(0)
    Qs = [torch.full((M, ldq), 1e-3, dtype=torch.float64, device="cuda") for _ in range(R)]
    Ks = [torch.zeros(M, dtype=torch.float64, device="cuda") for _ in range(R)]
    Vs = [torch.ones(B, M, dtype=torch.float64, device="cuda") for _ in range(R)]
    ms = lb.lindblad_time_stage(ctx, Qs, Ks, Vs, iters=2)
    log("copy 4 GiB done; stage GEMM %.3f ms per launch, %d systems, %d bytes of Q per launch"
        % (ms, R, R * M * M * 8))
    ctx.close()


def pmc_c3(args):
    """Kernels for the matrix-core counters of C3: the stage GEMM over C3's Q
    (N=100, M=9999, 64 states) launched 10 times in FP64 and 10 times in FP32."""
    import torch

    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, B = 100, 64
    M = N * N - 1
    H, gamma = wl.random_lindbladian(N, 0)
    ctx = lb.Context(0)
    Q, K = lb.lindblad_prepare(ctx, torch.from_numpy(H).cuda(), torch.from_numpy(gamma).cuda())
    Q32 = lb.lindblad_q_to_f32(ctx, Q)
    V = torch.zeros((B, M), dtype=torch.float64, device="cuda")
    out = {}
    for name, prec in (("fp64", lb.FP64), ("fp32", lb.FP32)):
        ms = lb.lindblad_time_stage(ctx, [Q] if prec == lb.FP64 else None, [K], [V], iters=10, precision=prec,
                                    Q32s=[Q32] if prec == lb.FP32 else None)
        out[name] = {"ms": ms, "tflops": 2.0 * M * M * B / ms / 1e9, "tile": lb.lindblad_tile_info(ctx, M, B, prec)}
        log("C3 stage GEMM %s: %.3f ms per launch, %.1f TFLOP/s" % (name, ms, out[name]["tflops"]))
    ctx.close()
    print(json.dumps(out), flush=True)


def pmc_assembly(args):
    """Kernels for the assembly's HBM traffic counters: a plain copy of 4 GiB
    (the scale for FETCH_SIZE / WRITE_SIZE), then one dense preparation at
    N (default 200) with gamma drawn beforehand (the draw's kernels are not
    the library's and are told apart by name)."""
    import torch

    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    n = 1 << 29  # doubles: 4 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    N = args.N
    ctx = lb.Context(0)
    H = torch.from_numpy(wl.gue_hamiltonian(N, 0)).cuda()
    gamma = wl.wishart_kossakowski_device(N, 1000, device="cuda")
    torch.cuda.synchronize()
    log("gamma drawn; preparing N=%d" % N)
    Q, K = lb.lindblad_prepare(ctx, H, gamma)
    ctx.sync()
    log("copy 4 GiB done; one preparation at N=%d done" % N)
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (--gpus %d requested)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        return pmc_probe(args)
    if args.pmc_assembly:
        return pmc_assembly(args)
    if args.pmc_c3:
        return pmc_c3(args)
    if args.serving or args.config in ("c5", "c5r"):
        return serving(args)
    if args.config in ("c1", "c2", "c2p", "c3", "c6", "c6s", "c7", "c8"):
        return {"c1": config_c1, "c2": config_c2, "c2p": config_c2p, "c3": config_c3, "c6": config_c6,
                "c6s": config_c6s, "c7": config_c7, "c8": config_c8}[args.config](args)
    return config_c4(args)


def config_c4(args):
    """The headline configuration: N = 200 dense random Lindbladians, 8
    realizations assembled once and held resident, 16 pure states each, one
    timed step = one batched RK4 step over the 8 x 16 states."""
    import numpy as np
    import torch

    import paper_1912_01491_amd as lb
    from paper_1912_01491_amd import workloads as wl

    N, R, B, dt = args.N, args.realizations, args.states, args.dt
    M = N * N - 1
    ldq = lb.default_ldq(M)
    prec = lb.FP32 if args.precision == "fp32" else lb.FP64
    K_steps, W_steps = (args.rk4_steps, 0) if args.full_job else (args.steps, args.warmup)
    want_cpu = not args.no_cpu_baseline
    dev = torch.device("cuda", 0)
    ctx = lb.Context(0)
    log("N=%d M=%d realizations=%d states=%d precision=%s: %d warmup + %d timed batched RK4 steps"
        % (N, M, R, B, args.precision, W_steps, K_steps))

    Hs = [torch.from_numpy(wl.gue_hamiltonian(N, r)).to(dev) for r in range(R)]
    psis = [torch.from_numpy(wl.random_pure_states(N, B, 100 + r)).to(dev) for r in range(R)]
    Qs = [torch.empty((M, ldq), dtype=torch.float64, device=dev) for _ in range(R)]
    Ks = [torch.empty(M, dtype=torch.float64, device=dev) for _ in range(R)]
    Q32s = [torch.empty((M, ldq), dtype=torch.float32, device=dev) for _ in range(R)] if prec == lb.FP32 else None

    # assembly: each realization once, gamma resident when the timer starts
    t_prep, t_prep_ev, t_draw = [], [], []
    gamma0_host = None
    psd = None
    for r in range(R):
        t = time.perf_counter()
        gamma = wl.wishart_kossakowski_device(N, 1000 + r, device=dev)
        torch.cuda.synchronize()
        t_draw.append(time.perf_counter() - t)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if r == 0:  # untimed warm-up: the library's first-use set-up (workspace, streams, code objects)
            lb.lindblad_prepare(ctx, Hs[r], gamma, ldq=ldq, Q=Qs[r], K=Ks[r])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        lb.lindblad_prepare(ctx, Hs[r], gamma, ldq=ldq, Q=Qs[r], K=Ks[r])
        e1.record()
        torch.cuda.synchronize()
        t_prep.append(time.perf_counter() - t0)
        t_prep_ev.append(e0.elapsed_time(e1) * 1e-3)
        if Q32s is not None:
            Q32s[r].copy_(lb.lindblad_q_to_f32(ctx, Qs[r]))
        if r == 0 and args.check_psd:
            _, info = torch.linalg.cholesky_ex(gamma)
            torch.cuda.synchronize()
            psd = {"cholesky_info": int(info.item()), "realization": 0}
            log("gamma of realization 0: Cholesky info %d (0 = positive definite to FP64 rounding)" % psd["cholesky_info"])
        if r == 0 and want_cpu:
            gamma0_host = gamma.cpu().numpy()
        del gamma
        torch.cuda.empty_cache()
        log("realization %d: gamma drawn in %.1f s, prepared in %.2f ms (%.2f ms HIP events)"
            % (r, t_draw[-1], 1e3 * t_prep[-1], 1e3 * t_prep_ev[-1]))

    if args.autotune:
        lb.lindblad_autotune(ctx, Qs[0] if prec == lb.FP64 else None, Ks[0], B, precision=prec,
                             Q32=Q32s[0] if Q32s else None)
        log("autotuned tile: %s" % lb.lindblad_tile_info(ctx, M, B, prec))
    Vs = [lb.lb_expand_pure(ctx, psis[r]) for r in range(R)]
    V0_host = Vs[0].cpu().numpy() if want_cpu else None
    torch.cuda.synchronize()

    def run(steps):
        if steps == 0:
            return
        if args.graph:
            for r in range(R):
                lb.lindblad_propagate_graph(ctx, Qs[r] if prec == lb.FP64 else None, Ks[r], Vs[r], dt, steps,
                                            precision=prec, Q32=Q32s[r] if Q32s else None)
        else:
            lb.lindblad_propagate_batched(ctx, Qs if prec == lb.FP64 else None, Ks, Vs, dt, steps, precision=prec,
                                          Q32s=Q32s)

    run(W_steps)
    torch.cuda.synchronize()
    log("%d warmup steps done; timing %d batched RK4 steps" % (W_steps, K_steps))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    run(K_steps)
    e1.record()
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t0
    t_events = e0.elapsed_time(e1) * 1e-3
    log("timed: %.3f s wall, %.3f s HIP events, %.2f ms per batched step" % (t_timed, t_events, 1e3 * t_timed / K_steps))
    value = R * K_steps / t_timed

    # checks on rho(t) after W + K steps: unit trace, Hermitian, positive
    rhos = [lb.lb_reconstruct(ctx, Vs[r], N) for r in range(R)]
    rho = torch.cat(rhos).cpu().numpy()
    tr_err = float(np.abs(np.einsum("bii->b", rho) - 1).max())
    herm = float(np.abs(rho - rho.conj().transpose(0, 2, 1)).max())
    mineig = float(min(np.linalg.eigvalsh(x).min() for x in rho))
    finite = bool(all(torch.isfinite(k).all().item() for k in Ks))

    # dominant kernel: RK4 stage GEMM over all R systems, HIP events on its stream
    Vt = [torch.zeros((B, M), dtype=torch.float64, device=dev) for _ in range(R)]
    avg_ms = lb.lindblad_time_stage(ctx, Qs if prec == lb.FP64 else None, Ks, Vt, iters=5, precision=prec,
                                    Q32s=Q32s)
    del Vt
    qbytes = 8 if prec == lb.FP64 else 4
    alg_bytes = R * M * M * qbytes
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    tile = lb.lindblad_tile_info(ctx, M, B, prec)
    log("stage GEMM: %.3f ms per launch over %d systems -> %.0f GB/s" % (avg_ms, R, achieved))

    t_prep_mean = sum(t_prep) / len(t_prep)
    asm_bytes = 16.0 * M * M  # independent reals of gamma + Q, 8 bytes each
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RK4 steps/s per 16-state block (N=200; %d blocks advanced per batched step)" % R,
        "n_gpus": 1,
        "steps": K_steps,
        "warmup": W_steps,
        "ms_per_step": 1e3 * t_timed / K_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == lb.FP64 else "f32-mfma/f64",
        "data": "synthetic",
        "config": {
            "workload": "dense random Lindbladian N=%d (M=%d), %d realizations x %d pure states resident, "
                        "one step = one batched RK4 step (dt=%g) over all of them" % (N, M, R, B, dt),
            "N": N, "M": M, "realizations": R, "states": B, "dt": dt, "full_job": bool(args.full_job),
            "precision": args.precision, "ldq": ldq, "graph": bool(args.graph), "tile": tile,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(M, R, B, tile) if prec == lb.FP64 else None,
            "kernel": ("k_gemm64" if prec == lb.FP64 else "k_gemm32")
                      + ("s" if staged(Qs if prec == lb.FP64 else Q32s, ldq, qbytes) else ""),
            "avg_ms": avg_ms,
            "bytes_per_launch": alg_bytes,
        },
        "timed_s_hip_events": t_events,
        "assembly_s_per_realization": t_prep_mean,
        "assembly_s_hip_events": sum(t_prep_ev) / len(t_prep_ev),
        "assembly_s_all": t_prep,
        "assembly_s_median": sorted(t_prep)[len(t_prep) // 2],
        "assembly_gbs": asm_bytes / t_prep_mean / 1e9,
        "assembly_frac_hbm": asm_bytes / t_prep_mean / 1e9 / HBM_PEAK_GBS,
        "assembly_roofline": {
            "bound": "hbm",
            "kernel": "k_quad (+ side kernels on a second stream)",
            "achieved": asm_bytes / t_prep_mean / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": asm_bytes / t_prep_mean / 1e9 / HBM_PEAK_GBS,
            "bytes_per_preparation": asm_bytes,
            "design_bytes": 24.0 * M * M,
            "traffic": assembly_traffic(N, M, ldq),
        },
        "gamma_draw_s": sum(t_draw) / len(t_draw),
        "solves_per_s": R * B / (t_prep_mean * R + t_timed / K_steps * args.rk4_steps),
        "checks": {"max_abs_trace_err": tr_err, "max_herm_err": herm, "min_eig_rho": mineig,
                   "K_finite": finite, "gamma_psd": psd},
    }
    # the device's read-stream rate, measured after the timed region: the practical ceiling
    # of the HBM-bound stage kernel next to the published peak
    Q0_host = np.ascontiguousarray(Qs[0].cpu().numpy()[:, :M]) if want_cpu else None
    K0_host = Ks[0].cpu().numpy() if want_cpu else None
    Qs.clear()
    if Q32s is not None:
        Q32s.clear()
    torch.cuda.empty_cache()
    read_gbs = lb.read_bandwidth(ctx, 4 << 30)
    out["roofline"]["measured_read_gbs"] = read_gbs
    out["roofline"]["frac_of_measured_read"] = achieved / read_gbs
    log("read-stream probe: %.0f GB/s; stage kernel at %.1f %% of it" % (read_gbs, 100.0 * achieved / read_gbs))
    if want_cpu:
        out["cpu_baseline"] = cpu_baseline(Q0_host, K0_host, V0_host, args.cpu_steps, N,
                                           H0=Hs[0].cpu().numpy(), gamma0=gamma0_host, nrows=args.cpu_rows)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
