"""Benchmark of the weak-lensing P+B covariance hot path on one MI355X.

One step = one pass of the whole path over the synthetic workload: wlc_run
(enumeration upload, table staging, halo-model quadrature and Limber
projection, A-build, one-halo Gram product, covariance assembly) followed by
wlc_snr2 (FP64 bordered Cholesky and S/N).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload large10|euclid5]
                  [--precision bf16_auto|bf16x3|bf16|fp32|fp64] [--fp64-steps S] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0, "bf16_auto": 2500.0, "fp32": 157.3, "fp64": 78.6}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large10")
    ap.add_argument("--precision", default="bf16_auto",
                    help="Gram precision of the headline step: bf16_auto (one bf16 product per tile where the "
                         "a-priori bound allows, the split product elsewhere), bf16x3, bf16, fp32 or fp64")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--chi-steps", type=int, default=1,
                    help="steps of the FP64 path with the one-halo term factorised along chi (0: skip)")
    ap.add_argument("--n-sub", type=int, default=3,
                    help="sub-bins per side of the bin-averaged leg (<= 1 skips it)")
    ap.add_argument("--pca-workload", default="euclid5",
                    help="workload of the PCA leg (FP64 covariance, then wlc_pca; empty: skip)")
    ap.add_argument("--pca-only", action="store_true")
    ap.add_argument("--pca-tomography", action="store_true",
                    help="also run the PCA of the paper's 14-bin binning with 1, 2 and 5 redshift bins")
    ap.add_argument("--precision-workload", default="euclid5",
                    help="workload of the Gram precision report (bf16, bf16x3, fp32 vs FP64; empty: skip)")
    ap.add_argument("--no-gram-variants", dest="gram_variants", action="store_false",
                    help="skip timing the plain bf16 and FP32 Gram on the bench workload")
    ap.add_argument("--lattice-workload", default="euclid5",
                    help="workload of the timed lattice counts (empty: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-requests", type=int, default=8,
                    help="requests of the serving stream (0: skip serving)")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-budget-gb", type=float, default=180.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-snr", default="direct,structured",
                    help="S/N methods of the serving legs: direct (Cholesky of the whole covariance) and/or "
                         "structured (through the distinct rows)")
    ap.add_argument("--no-serve-fp64", action="store_true",
                    help="serve the stream in the headline precision only (default: also the plain FP64 path)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (to scale HBM byte counters)")
    return ap.parse_args()


def measured_traffic(*names, per=None):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the record
    is missing or the kernel's source has changed since the counters were
    taken.  Several names are summed over their launches and divided by the
    launches of those named in per (default: the first), e.g. a kernel and
    its helper timed as one launch."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    total = 0.0
    for n in names:
        r = rec.get(n)
        if r is None or r.get("fetch_bytes_per_launch") is None or r.get("write_bytes_per_launch") is None:
            return None
        h = hashlib.sha256()
        for src in r["source"].split("+"):  # several sources hash as one text
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != r["source_sha256"]:
            return None
        total += (r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"]) * r["launches"]
    launches = sum(rec[n]["launches"] for n in (per or names[:1]))
    return dict(bytes_per_launch=total / launches, summary=rec[names[0]]["summary"])


def gram_flops(n_r, k_len):
    """Flops of the flattened one-halo Gram: each of the n_r (n_r + 1)/2
    distinct entries as a length-K dot product (2K flops)."""
    return n_r * (n_r + 1) * k_len


def gram_figures(ms, n_r, k_len, precision, work, split=None):
    """Gram rates against the peak of the precision's matrix-core type.
    work = (flops, MFMA flops) the product did (wlc_gram_work: the bf16
    products sum each tile only up to the column where the shorter of its two
    panels' factors ends, the split tiles count three times in the second).
    dense_equivalent_tflops: the flattened product's flops N_R (N_R + 1) K
    over the time, i.e. as if every column were summed (it can exceed the
    peak); executed_tflops and mfma_work_tflops: the flops done.  split =
    (tiles with the split product, tiles) for the per-tile precision."""
    t = ms * 1e-3
    dense = gram_flops(n_r, k_len) / t / 1e12
    executed, mfma = work[0] / t / 1e12, work[1] / t / 1e12
    peak = PEAK_TFLOPS[precision]
    out = dict(ms=ms, dense_equivalent_tflops=dense, executed_tflops=executed, frac_peak_executed=executed / peak,
               mfma_work_tflops=mfma, frac_peak_mfma_work=mfma / peak, peak_tflops=peak,
               executed_fraction_of_dense=work[0] / max(gram_flops(n_r, k_len), 1.0))
    if split:
        out["split_tiles"], out["tiles"] = split
    return out


def timed_runs(prob, runs, warmup, torch, wl):
    """Phase times of wlc_run alone (no S/N), averaged over runs."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        prob.run(stream)
    torch.cuda.synchronize()
    wl.wlc_plan_set_timing(prob.plan, True)
    phases = {p: 0.0 for p in wl.PHASES}
    for _ in range(runs):
        prob.run(stream)
        for k, v in wl.wlc_plan_timings(prob.plan).items():
            phases[k] += v
    torch.cuda.synchronize()
    wl.wlc_plan_set_timing(prob.plan, False)
    return {k: v / runs for k, v in phases.items()}


def true_cov(prob, torch):
    """C_true = C 2^-(t_a + t_b) on the device, float64."""
    t = prob.row_exp2.to(torch.int64)
    return torch.ldexp(prob.C.double(), -(t[:, None] + t[None, :]).double())


def precision_report(workload, torch, wl):
    """The Gram precisions at one workload (the Euclid-like shape by
    default): bf16, split bf16 x 3, the per-tile choice and FP32 against the FP64 path on the same
    tables -- Gram time, its rate on the flops done against peak, its dense-equivalent rate,
    diagonal max / median relative error, off-diagonal error relative to
    sqrt(C_aa C_bb), and the (S/N)^2 error -- and for each precision the
    whole step (wlc_run and the direct S/N) in ms with the unique covariance
    entries per second."""
    import synth
    t = synth.make_tables(workload)
    out = {"workload": workload}
    p64 = wl.Problem(t.cfg, t.arrays(), precision="fp64", device="cuda:0")
    s = p64.sizes
    NR, K = s.n_distinct, s.k_len
    N = s.n_data
    entries = N * (N + 1) / 2

    def step_figures(prob):
        dt, _, _, _ = timed_steps(prob, 3, 1, torch, wl)
        return dict(step_ms=dt / 3 * 1e3, entries_per_s=entries / (dt / 3))

    ph = timed_runs(p64, 2, 1, torch, wl)
    snr64 = p64.snr2()
    C64 = true_cov(p64, torch)
    d64 = torch.diagonal(C64).clone()
    out["fp64"] = dict(gram=gram_figures(ph["gram"], NR, K, "fp64", p64.gram_work()), snr2=snr64,
                       **step_figures(p64))
    log("precision %s fp64: step %.2f ms (%.3g entries/s), gram %.3f ms" % (
        workload, out["fp64"]["step_ms"], out["fp64"]["entries_per_s"], ph["gram"]))
    del p64
    scale = torch.sqrt(torch.outer(d64, d64))
    for prec in ("bf16", "bf16x3", "bf16_auto", "fp32"):
        pm = wl.Problem(t.cfg, t.arrays(), precision=prec, device="cuda:0")
        ph = timed_runs(pm, 2, 1, torch, wl)
        split = pm.split_tiles() if prec == "bf16_auto" else None
        snr = pm.snr2()
        Cm = true_cov(pm, torch)
        dm = torch.diagonal(Cm)
        ed = torch.abs(dm - d64) / d64
        off = torch.abs(Cm - C64) / scale
        off.fill_diagonal_(0.0)
        out[prec] = dict(gram=gram_figures(ph["gram"], NR, K, prec, pm.gram_work(), split),
                         diag_max_rel=float(ed.max()),
                         diag_median_rel=float(ed.median()), offdiag_max_rel_sqrt_caa_cbb=float(off.max()),
                         snr2_rel=abs(snr - snr64) / snr64, **step_figures(pm))
        log("precision %s %s: step %.2f ms, gram %.3f ms (%.1f %% of peak on the flops done), diag max %.2e "
            "median %.2e, off %.2e, snr %.2e" % (workload, prec, out[prec]["step_ms"], ph["gram"],
                                                 100 * out[prec]["gram"]["frac_peak_mfma_work"],
                                                 out[prec]["diag_max_rel"], out[prec]["diag_median_rel"],
                                                 out[prec]["offdiag_max_rel_sqrt_caa_cbb"], out[prec]["snr2_rel"]))
        del pm, Cm, off
        torch.cuda.empty_cache()
    del C64, scale
    torch.cuda.empty_cache()
    return out


def gram_variants(cfg, arrays, torch, wl, precisions):
    """Gram time of the other precisions on the bench workload (wlc_run
    only, one warm-up and one timed run each)."""
    out = {}
    for prec in precisions:
        p = wl.Problem(cfg, arrays, precision=prec, device="cuda:0")
        s = p.sizes
        ph = timed_runs(p, 1, 1, torch, wl)
        out[prec] = gram_figures(ph["gram"], s.n_distinct, s.k_len, prec, p.gram_work(),
                                 p.split_tiles() if prec == "bf16_auto" else None)
        out[prec]["run_ms"] = sum(ph[k] for k in ("tables", "abuild", "gram", "assemble"))
        log("gram %s: %.1f ms, %.1f TFLOP/s of MFMA work (%.1f %% of its peak), dense-equivalent %.1f TFLOP/s" % (
            prec, ph["gram"], out[prec]["mfma_work_tflops"], 100 * out[prec]["frac_peak_mfma_work"],
            out[prec]["dense_equivalent_tflops"]))
        del p
        torch.cuda.empty_cache()
    return out


def lattice_leg(workload, torch, wl, reps=3):
    """Integer lattice counts of modes and triangles (wlc_lattice_counts)
    on a workload's binning, timed with events on the launch stream."""
    import synth
    t = synth.make_tables(workload)
    p = wl.Problem(t.cfg, t.arrays(), precision="fp64_chi", device="cuda:0")
    stream = torch.cuda.current_stream()
    p.lattice_counts(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        modes, tris = p.lattice_counts(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out = dict(workload=workload, ms=ms, n_tri=int(p.sizes.n_tri), n_ell=int(p.sizes.n_ell_used),
               modes_total=int(modes.sum()), pairs_total=int(tris.sum()))
    log("lattice counts %s: %.2f ms (%d triangles, %.3e mode pairs)" % (workload, ms, out["n_tri"],
                                                                        out["pairs_total"]))
    del p
    return out


def pca_leg(args, torch, wl):
    """Principal components (Sec. 6) of the FP64 joint covariance of the
    Euclid-like workload: eigenvalues over tens of decades, per-mode and
    cumulative S/N, the share of modes holding 99 % of (S/N)^2 and the
    observables with |S_ai| >= 0.05 in the modes holding 95 %."""
    import numpy as np
    import synth
    log("pca on %s (FP64 covariance)" % args.pca_workload)
    tp = synth.make_tables(args.pca_workload)
    pp = wl.Problem(tp.cfg, tp.arrays(), precision="fp64", device="cuda:0")
    pp.run()
    snr_p = pp.snr2()
    torch.cuda.synchronize()
    pp.free_snr_workspace()
    pp.pca(vectors=True)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, snr_m, cum, sweeps, S = pp.pca(vectors=True)
    torch.cuda.synchronize()
    t_pca = time.perf_counter() - t0
    t0 = time.perf_counter()
    pp.pca(vectors=False)
    torch.cuda.synchronize()
    t_pca_nov = time.perf_counter() - t0
    npca = len(lam)
    k99 = int(np.searchsorted(cum, 0.99 * cum[-1]) + 1)
    k95 = int(np.searchsorted(cum, 0.95 * cum[-1]) + 1)
    top95 = torch.as_tensor(np.argsort(-snr_m, kind="stable")[:k95], device=S.device)
    involved = int(torch.count_nonzero(torch.any(torch.abs(S[top95]) >= 0.05, dim=0)).item())
    pca = dict(workload=args.pca_workload, n=npca, seconds=t_pca, seconds_without_vectors=t_pca_nov,
               sweeps=sweeps, lambda_min=float(lam[0]), lambda_max=float(lam[-1]),
               decades=float(np.log10(lam[-1] / lam[0])), snr2_total=float(cum[-1]),
               snr2_rel_vs_cholesky=abs(cum[-1] - snr_p) / snr_p,
               modes_for_99pct=k99, frac_modes_for_99pct=k99 / npca, modes_for_95pct=k95,
               observables_in_95pct_modes=involved,
               flops_per_sweep_est=12.0 * (((npca + 63) // 64) * 64) ** 3)
    log("pca %s: N=%d, %.2f s (%.2f s without vectors), %d sweeps, lambda %.2e..%.2e (%.1f decades), "
        "99%% of (S/N)^2 in %d modes (%.1f %%), %d observables in the 95%% modes" % (
            args.pca_workload, npca, t_pca, t_pca_nov, sweeps, lam[0], lam[-1], pca["decades"], k99,
            100.0 * k99 / npca, involved))
    del S, pp
    torch.cuda.empty_cache()
    # the paper's PCA study: its 14 ell-bins over 10-5000 with 1, 2 and 5
    # redshift bins (joint vectors of 144, 818 and 10000 rows); the share of
    # modes holding 99 % of (S/N)^2 as the tomography grows
    if args.pca_tomography:
        rows = []
        for nz in (1, 2, 5):
            tz = synth.make_tables("paper14", n_z=nz)
            pz = wl.Problem(tz.cfg, tz.arrays(), precision="fp64", device="cuda:0")
            pz.run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lz, sz, cz, swz, _ = pz.pca(vectors=False)
            torch.cuda.synchronize()
            dtz = time.perf_counter() - t0
            k = int(np.searchsorted(cz, 0.99 * cz[-1]) + 1)
            rows.append(dict(n_z=nz, n=len(lz), seconds=dtz, sweeps=swz, decades=float(np.log10(lz[-1] / lz[0])),
                             modes_for_99pct=k, frac_modes_for_99pct=k / len(lz)))
            log("pca paper binning n_z=%d: N=%d, %.2f s, %d sweeps, %.1f decades, 99%% of (S/N)^2 in %d modes "
                "(%.1f %%)" % (nz, len(lz), dtz, swz, rows[-1]["decades"], k, 100.0 * k / len(lz)))
            del pz
            torch.cuda.empty_cache()
        pca["paper_tomography"] = rows
    return pca


def timed_steps(prob, steps, warmup, torch, wl, structured=False):
    """Time whole steps (run + S/N); structured=True takes the S/N through
    the distinct rows instead of the Cholesky of the whole covariance."""
    stream = torch.cuda.current_stream()
    snr = prob.snr2_structured if structured else prob.snr2
    for _ in range(warmup):
        prob.run(stream)
        snr(stream)
    torch.cuda.synchronize()
    wl.wlc_plan_set_timing(prob.plan, True)
    phases = {p: 0.0 for p in wl.PHASES}
    upd = dict(ms=0.0, launches=0, timed=0, flops=0.0)
    t_snr = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.run(stream)
        s = snr(stream)
        t_snr.append(s)
        ph = wl.wlc_plan_timings(prob.plan)
        for k, v in ph.items():
            phases[k] += v
        ks = wl.wlc_plan_kernel_stats(prob.plan)
        for k in upd:
            upd[k] += ks[k]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    wl.wlc_plan_set_timing(prob.plan, False)
    upd = {k: v / steps for k, v in upd.items()}
    return dt, {k: v / steps for k, v in phases.items()}, t_snr, upd


def cpu_baseline(tables, seconds, n_data):
    """The oracle as it stands on the host cores: data vector for every row,
    then covariance entries on seeded row pairs, as many as fit in the time
    budget; entries/s from the pairs, with the data-vector time amortised the
    way one step amortises it."""
    import numpy as np
    import oracle
    import synth
    o = oracle.Oracle(tables)
    t0 = time.perf_counter()
    o.data_vector()
    o.u_table()
    t_setup = time.perf_counter() - t0
    n = 64
    done, t_pairs = 0, 0.0
    while t_pairs < seconds and done < 10 ** 7:
        pairs = synth.sample_pairs(o.N, n, seed=100 + done)
        t1 = time.perf_counter()
        o.cov_pairs(pairs)
        t_pairs += time.perf_counter() - t1
        done += n
        n = min(n * 2, 1 << 16)
    per_entry = t_pairs / done
    total = n_data * (n_data + 1) / 2
    est_step = t_setup + per_entry * total
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=total / est_step, unit="cov entries/s", cores=cores, kind="oracle",
                sample="data vector + %d seeded covariance entries (%.1f s); S/N Cholesky not included" %
                (done, t_setup + t_pairs))


def serve_precisions(args):
    """The headline precision, then the plain FP64 path for comparison."""
    return [args.precision] + ([] if args.no_serve_fp64 or args.precision == "fp64" else ["fp64"])


def serving(n_req, budget_gb, slots, precisions, torch, fractions=(0.5, 0.8), snr="direct"):
    """The request server on a seeded stream of requests (Omega_m, sigma_8,
    n_z, l_max drawn per request).  Closed loop first (every request
    submitted at once) for the capacity, then open loops with Poisson
    arrivals at the given fractions of it.  Each request's lensing kernels
    are built by the client when it arrives, so a request's latency runs
    from its arrival through that build, submission, queueing and the
    server's work to its completion.  Finished requests are released as soon
    as they are seen done, so the arena holds only live requests."""
    import numpy as np
    import synth
    from paper_1812_07437_amd import serve
    fid = synth.serving_fiducial()
    reqs = synth.serving_requests(n_req, seed=1234, qps=1.0, fid=fid)
    out = {"requests": n_req, "slots": slots, "arena_gb": budget_gb, "snr_method": snr,
           "mix": {"n_z": [int(q["n_z"]) for q in reqs], "ell_max": [q["ell_max"] for q in reqs]}}

    def build_w(q):
        return synth.lensing_kernels(fid.chi, q["omega_m"], synth.equipopulated_edges(q["n_z"]))

    def run_stream(srv, arrivals, label):
        """Submit request i at arrivals[i] (seconds from start; None = at once);
        returns per-request latency (s), queue time (s) and the wall time."""
        live = {}  # ticket -> (index, client delay before submission)
        lat = np.zeros(n_req)
        queue = np.zeros(n_req)
        ok = True
        done = 0
        t0 = time.perf_counter()

        def reap(block):
            nonlocal done, ok
            for t in list(live):
                fin, r = srv.poll(t)
                if not fin:
                    continue
                i, client = live.pop(t)
                lat[i] = client + (r.t_done_ms - r.t_submit_ms) * 1e-3
                queue[i] = (r.t_admit_ms - r.t_submit_ms) * 1e-3
                ok &= r.status == 0
                srv.release(t)
                done += 1
                if done % 10 == 0 or done == n_req:
                    log("  %s: %d/%d done at %.1f s" % (label, done, n_req, time.perf_counter() - t0))
            if block and live:
                time.sleep(0.0005)

        for i, q in enumerate(reqs):
            ta = arrivals[i] if arrivals is not None else 0.0
            while time.perf_counter() - t0 < ta:
                reap(False)
                time.sleep(0.0002)
            W = build_w(q)
            t = srv.submit(W, q["n_z"], q["ell_max"], q["p_scale"], q["n_scale"], q["rho_mean"], snr=snr)
            live[t] = (i, time.perf_counter() - t0 - ta)
        while live:
            reap(True)
        return lat, queue, time.perf_counter() - t0, ok

    for prec in precisions:
        srv = serve.Server(fid.cfg, fid.arrays(), hbm_budget=int(budget_gb * (1 << 30)), max_inflight=slots,
                           precision=prec)
        st0 = srv.stats()
        lat, _, t_closed, ok = run_stream(srv, None, "closed loop %s" % prec)
        cap = n_req / t_closed
        res = dict(closed_loop_req_per_s=cap, closed_loop_s=t_closed, all_ok=ok)
        log("serve %s: closed loop %d requests in %.1f s (%.2f req/s)" % (prec, n_req, t_closed, cap))
        for f in fractions:
            qps = f * cap
            arrivals = np.cumsum(np.random.default_rng(1234).exponential(1.0 / qps, size=n_req))
            lat, queue, t_open, ok = run_stream(srv, arrivals, "open loop %s at %.0f%%" % (prec, 100 * f))
            key = "open_%d" % round(100 * f)
            res[key] = dict(fraction_of_capacity=f, qps=qps, achieved_req_per_s=n_req / t_open, n=n_req,
                            p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                            max_ms=float(lat.max() * 1e3), mean_queue_ms=float(queue.mean() * 1e3), all_ok=ok)
            log("serve %s at %.0f%% (%.2f qps): p50 %.0f ms p99 %.0f ms (n = %d), mean queue %.0f ms" % (
                prec, 100 * f, qps, res[key]["p50_ms"], res[key]["p99_ms"], n_req, res[key]["mean_queue_ms"]))
        st = srv.stats()
        res.update(batches=st.batches - st0.batches, batched_requests=st.batched_requests - st0.batched_requests,
                   max_batch=st.max_batch, arena_peak_gb=st.arena_peak / 2 ** 30)
        srv.close()
        out[prec] = res
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the covariance and "
              "its Cholesky run on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1812_07437_amd import wlcov as wl

    if args.pca_only:
        print(json.dumps({"metric": "principal components of the joint covariance", "data": "synthetic",
                          "pca": pca_leg(args, torch, wl)}), flush=True)
        return

    if args.serve_only:
        srv = {m: serving(args.serve_requests, args.serve_budget_gb, args.serve_slots, serve_precisions(args), torch,
                          snr=m) for m in args.serve_snr.split(",") if m}
        print(json.dumps({"metric": "serving p50/p99 latency (ms) and requests/s", "data": "synthetic",
                          "serving": srv}), flush=True)
        return

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst

    log("building %s tables" % args.workload)
    t = synth.make_tables(args.workload)
    cfg = t.cfg
    prob = wl.Problem(cfg, t.arrays(), precision=args.precision, device="cuda:0")
    s = prob.sizes
    N, NR, K = s.n_data, s.n_distinct, s.k_len
    log("N=%d N_R=%d K=%d precision=%s" % (N, NR, K, args.precision))
    dt, ph, snrs, upd = timed_steps(prob, args.steps, args.warmup, torch, wl)
    ms_step = dt / args.steps * 1e3
    entries = N * (N + 1) / 2
    value = entries / (dt / args.steps)
    log("mixed: %.1f ms/step  phases %s  snr2 %.6e" % (ms_step, {k: round(v, 2) for k, v in ph.items()}, snrs[-1]))

    split_main = prob.split_tiles() if args.precision == "bf16_auto" else None
    work_main = prob.gram_work()
    d_mixed = prob.C.diagonal().double().cpu().numpy()
    t_mixed = prob.row_exp2.cpu().numpy().astype(np.int64)
    diag_mixed = np.ldexp(d_mixed, -2 * t_mixed)
    snr_mixed = snrs[-1]
    del prob
    torch.cuda.empty_cache()

    # plain FP64 GPU path on the same workload (reference for accuracy and speedup)
    fp64 = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        log("fp64 path")
        p64 = wl.Problem(cfg, t.arrays(), precision="fp64", device="cuda:0")
        dt64, ph64, snr64, _ = timed_steps(p64, args.fp64_steps, 1, torch, wl)
        work64 = p64.gram_work()
        d64 = p64.C.diagonal().cpu().numpy()
        t64 = p64.row_exp2.cpu().numpy().astype(np.int64)
        diag64 = np.ldexp(d64, -2 * t64)
        err_diag = float(np.max(np.abs(diag_mixed - diag64) / diag64))
        err_snr = float(abs(snr_mixed - snr64[-1]) / snr64[-1])
        fp64 = dict(ms_per_step=dt64 / args.fp64_steps * 1e3, value=entries / (dt64 / args.fp64_steps),
                    phases_ms=ph64, speedup_step=(dt64 / args.fp64_steps) / (dt / args.steps),
                    speedup_gram=ph64["gram"] / max(ph["gram"], 1e-9),
                    gram=gram_figures(ph64["gram"], NR, K, "fp64", work64),
                    err_vs_fp64={"diag_max_rel": err_diag, "snr2_rel": err_snr})
        log("fp64: %.1f ms/step  gram %.1f ms  diag err %.2e  snr err %.2e" % (fp64["ms_per_step"], ph64["gram"],
                                                                           err_diag, err_snr))
        fp64["snr2"] = snr64[-1]
        del p64
        torch.cuda.empty_cache()

    others = [q for q in ("bf16", "bf16x3", "bf16_auto", "fp32") if q != args.precision]
    variants = gram_variants(cfg, t.arrays(), torch, wl, others) if args.gram_variants else None
    prec_rep = precision_report(args.precision_workload, torch, wl) if args.precision_workload else None
    lattice = lattice_leg(args.lattice_workload, torch, wl) if args.lattice_workload else None

    # FP64 path with the one-halo sum taken over M first and chi second
    # (exact; N_M times fewer one-halo operations than the flattened Gram)
    chi = None
    if args.chi_steps > 0:
        log("fp64 chi-factorised path")
        pc = wl.Problem(cfg, t.arrays(), precision="fp64_chi", device="cuda:0")
        dtc, phc, snrc, _ = timed_steps(pc, args.chi_steps, 1, torch, wl)
        n_cfg = int(pc.sizes.n_cfg)
        chi_flops = NR * (NR + 1) * cfg["n_chi"] + 2.0 * n_cfg * n_cfg * cfg["n_chi"] * cfg["n_m"]
        ref_snr = fp64["snr2"] if fp64 else snr_mixed
        chi = dict(ms_per_step=dtc / args.chi_steps * 1e3, value=entries / (dtc / args.chi_steps), phases_ms=phc,
                   one_halo_ms=phc["gram"], one_halo_tflops=chi_flops / (phc["gram"] * 1e-3) / 1e12,
                   one_halo_speedup_vs_mixed_gram=ph["gram"] / max(phc["gram"], 1e-9),
                   snr2_rel_vs=("fp64" if fp64 else args.precision), snr2_rel=abs(snrc[-1] - ref_snr) / ref_snr)
        log("fp64 chi: %.1f ms/step  one-halo %.2f ms  snr rel %.2e" % (chi["ms_per_step"], phc["gram"],
                                                                      chi["snr2_rel"]))
        # the same step with the S/N through the distinct rows
        pc.free_snr_workspace()
        dts, phs, snrs_, _ = timed_steps(pc, args.chi_steps, 1, torch, wl, structured=True)
        chi["structured"] = dict(ms_per_step=dts / args.chi_steps * 1e3, value=entries / (dts / args.chi_steps),
                                 phases_ms=phs, snr2_rel=abs(snrs_[-1] - ref_snr) / ref_snr,
                                 speedup_vs_headline_step=(dt / args.steps) / (dts / args.chi_steps))
        log("fp64 chi + structured S/N: %.1f ms/step  phases %s  snr rel %.2e" % (
            chi["structured"]["ms_per_step"], {k: round(v, 2) for k, v in phs.items()}, chi["structured"]["snr2_rel"]))
        del pc
        torch.cuda.empty_cache()

    # the same FP64 step with the B.B, P.T and P.B in-survey terms added
    ngins = None
    if args.chi_steps > 0:
        log("fp64 chi path with the B.B, P.T, P.B terms")
        pn = wl.Problem(cfg, t.arrays(), precision="fp64_chi", device="cuda:0", ngins=True)
        try:
            dtn, phn, snrn, _ = timed_steps(pn, args.chi_steps, 1, torch, wl)
            ngins = dict(ms_per_step=dtn / args.chi_steps * 1e3, phases_ms=phn, snr2=snrn[-1],
                         snr2_without=(fp64["snr2"] if fp64 else snr_mixed))
            log("fp64 chi + in-survey terms: %.1f ms/step  phases %s  (S/N)^2 %.6e (without: %.6e)" % (
                ngins["ms_per_step"], {k: round(v, 2) for k, v in phn.items()}, snrn[-1], ngins["snr2_without"]))
        except wl.WlcError as e:
            # the printed B.B / P.B terms need not keep the covariance positive
            # definite; report the run time and the failure
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pn.run(torch.cuda.current_stream())
            torch.cuda.synchronize()
            ngins = dict(run_ms=(time.perf_counter() - t0) * 1e3, snr2=None, error=str(e))
            log("fp64 chi + in-survey terms: run %.1f ms; S/N: %s" % (ngins["run_ms"], e))
        del pn
        torch.cuda.empty_cache()

    # the FP64 step with the super-sample term resolved along chi (sigma_W^2
    # of the survey disk), S/N through the distinct rows
    sscc = None
    if args.chi_steps > 0:
        log("fp64 chi path with the chi-resolved super-sample term")
        ps = wl.Problem(cfg, t.arrays(), precision="fp64_chi", device="cuda:0", ssc_chi=True)
        dtx, phx, snrx, _ = timed_steps(ps, args.chi_steps, 1, torch, wl, structured=True)
        ref_snr = fp64["snr2"] if fp64 else snr_mixed
        sw = ps.sigma_w2().cpu().numpy()
        sscc = dict(ms_per_step=dtx / args.chi_steps * 1e3, phases_ms=phx, snr2=snrx[-1], snr2_rank_one=ref_snr,
                    sigma_w2_range=[float(sw.min()), float(sw.max())])
        log("fp64 chi + chi-resolved SSC (structured S/N): %.1f ms/step  phases %s  (S/N)^2 %.6e (rank-one: %.6e)"
            % (sscc["ms_per_step"], {k: round(v, 2) for k, v in phx.items()}, snrx[-1], ref_snr))
        del ps
        torch.cuda.empty_cache()

    # the FP64 step with every polyspectrum averaged over 3 x 3 sub-bins per
    # bin (the average the paper replaces by the bin centres)
    subbin = None
    if args.chi_steps > 0 and args.n_sub > 1:
        log("fp64 chi path with bin averaging (n_sub=%d)" % args.n_sub)
        pb = wl.Problem(cfg, t.arrays(), precision="fp64_chi", device="cuda:0", n_sub=args.n_sub)
        dtb, phb, snrb, _ = timed_steps(pb, args.chi_steps, 1, torch, wl, structured=True)
        ref_snr = fp64["snr2"] if fp64 else snr_mixed
        subbin = dict(n_sub=args.n_sub, n_avg=int(pb.sizes.n_avg), ms_per_step=dtb / args.chi_steps * 1e3,
                      phases_ms=phb, snr2=snrb[-1], snr2_bin_centres=ref_snr)
        log("fp64 chi + bin averaging (structured S/N): %.1f ms/step  phases %s  (S/N)^2 %.6e (centres: %.6e)" % (
            subbin["ms_per_step"], {k: round(v, 2) for k, v in phb.items()}, snrb[-1], ref_snr))
        del pb
        torch.cuda.empty_cache()

    pca = pca_leg(args, torch, wl) if args.pca_workload else None

    # roofline of the dominant kernel of the step: the one-halo Gram (one
    # launch per step) or the Cholesky block update (many launches per step,
    # timed one by one with HIP events on the run's stream)
    gram_fig = gram_figures(ph["gram"], NR, K, args.precision, work_main, split_main)
    chol_flops = N ** 3 / 3.0
    chol_tf = chol_flops / (ph["chol"] * 1e-3) / 1e12
    upd_frac_timed = upd["timed"] / max(upd["launches"], 1)
    upd_ms = upd["ms"] / max(upd_frac_timed, 1e-9)
    upd_tf = upd["flops"] / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else 0.0
    if upd_ms >= ph["gram"]:
        # every block update is timed, on 128 x 256 tiles (k_update2d) or
        # 128 x 128 ones (k_update2<4>), with its split-k reduction
        tr = measured_traffic("k_update2d", "k_update2", "k_update_reduce", per=("k_update2d", "k_update2"))
        roof = dict(bound="mfma", kernel="k_update2d + k_update2<4> (FP64 Cholesky block update, incl. split-k "
                    "reduce)",
                    achieved=upd_tf, peak=PEAK_TFLOPS["fp64"], unit="TFLOP/s", frac=upd_tf / PEAK_TFLOPS["fp64"],
                    traffic=tr["bytes_per_launch"] / 1e9 if tr else None, launches=upd["launches"],
                    avg_launch_ms=upd_ms / max(upd["launches"], 1), flops_per_step=upd["flops"])
    else:
        tr = measured_traffic("k_gram_bf16")
        roof = dict(bound="mfma", kernel="k_gram_bf16 (one-halo Gram, MFMA flops done)",
                    achieved=gram_fig["mfma_work_tflops"], peak=PEAK_TFLOPS[args.precision], unit="TFLOP/s",
                    frac=gram_fig["frac_peak_mfma_work"], traffic=tr["bytes_per_launch"] / 1e9 if tr else None,
                    launches=1, avg_launch_ms=ph["gram"], flops_per_step=work_main[1])
    roof["traffic_unit"] = "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["traffic_source"] = tr["summary"] if tr else None
    # the factor's bytes over the distinct rows: the bf16 factors up to each
    # panel's extent, with the lo half only where a tile can take the split
    a_bytes = work_main[2]
    c_bytes = N * N * (8 if args.precision == "fp64" else 4)
    kernels = dict(
        gram=gram_fig,
        abuild=dict(ms=ph["abuild"], gbs=a_bytes / (ph["abuild"] * 1e-3) / 1e9,
                    frac_hbm=a_bytes / (ph["abuild"] * 1e-3) / 1e9 / HBM_PEAK_GBS),
        assemble=dict(ms=ph["assemble"], gbs=c_bytes / (ph["assemble"] * 1e-3) / 1e9,
                      frac_hbm=c_bytes / (ph["assemble"] * 1e-3) / 1e9 / HBM_PEAK_GBS),
        chol=dict(ms=ph["chol"], tflops=chol_tf, frac_peak=chol_tf / PEAK_TFLOPS["fp64"]),
        chol_update=dict(ms=upd_ms, launches=upd["launches"], tflops=upd_tf, frac_peak=upd_tf / PEAK_TFLOPS["fp64"]),
    )

    srv = None
    if args.serve_requests > 0:
        log("serving stream (%d requests)" % args.serve_requests)
        srv = {m: serving(args.serve_requests, args.serve_budget_gb, args.serve_slots, serve_precisions(args), torch,
                          snr=m) for m in args.serve_snr.split(",") if m}

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, ~%.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(t, args.cpu_seconds, N)

    out = {
        "metric": "cov entries/s (joint P+B covariance incl. S/N) + %MFMA peak, mixed vs plain FP64",
        "value": value, "unit": "cov entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": "%s: n_z=%d, %d ell-bins %g-%g, N_chi=%d, N_M=%d (K=%d), N=%d, N_R=%d" %
                   (args.workload, cfg["n_z"], cfg["n_ell"], cfg["ell_min"], cfg["ell_max"], cfg["n_chi"],
                    cfg["n_m"], K, N, NR), "precision": args.precision, "parallelism": "none (1 GPU)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "phases_ms": ph,
        "kernels": kernels,
        "distinct_entries_per_s": NR * (NR + 1) / 2 / (dt / args.steps),
        "snr": math.sqrt(snr_mixed) if snr_mixed > 0 else None,
        "fp64_path": fp64,
        "gram_variants": variants,
        "precision_report": prec_rep,
        "lattice": lattice,
        "fp64_chi_path": chi,
        "fp64_chi_ngins_path": ngins,
        "fp64_chi_ssc_chi_path": sscc,
        "fp64_chi_subbin_path": subbin,
        "pca": pca,
        "serving": srv,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
