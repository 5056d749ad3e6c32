#!/usr/bin/env python3
"""Benchmark of the CF-completion hot path on one MI355X.

Workload (one step): batched fold-in of 1,000,000 new applications, each with 4..24
observed settings out of 480 (24 CPU caps x 20 GPU caps), against fixed 480 x 32 float32
setting factors (rank 32, weighted lambda = 0.05), through libopen's C ABI.  Inputs are
synthetic and already resident in HBM when the timed region starts.

Printed: one JSON line with the throughput in rows/s, the roofline of the dominant kernel
(live HIP-event timing of every kernel the library launches), the FP64 CPU oracle timed on
a bounded sample of the same rows, and the prediction RMSE of both against the noiseless
truth on unobserved entries.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 (vector and matrix)
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA


def dual_flops(n, k):
    # Gram n(n+1)k (symmetric), LDL^T/Cholesky n^3/3, two triangular solves 2n^2, output 2nk
    return n * (n + 1) * k + n ** 3 / 3.0 + 2 * n * n + 2 * n * k


def primal_flops(n, k):
    return n * k * (k + 1) + 2 * n * k + k ** 3 / 3.0 + 2 * k * k


def row_flops(n, k):
    import numpy as np
    n = np.asarray(n, dtype=np.float64)
    dual = n <= min(k, 32)
    return np.where(n == 0, 0.0, np.where(dual, dual_flops(n, k), primal_flops(n, k)))


def kernel_of_counts(n, k, mode=1):
    """Name of the ridge kernel that solves a row with n observations (matches the library):
    one launch per class group (mode 1): dual rows of n <= min(k, 32) go to the kernel of
    padded dimension 4 ceil(n/4), longer rows to the primal kernel; the merged launches of rank
    32 (mode 0): up to 12, 13-24, from 25 observations."""
    import numpy as np
    n = np.asarray(n)
    if k == 32 and mode == 0:
        out = np.full(n.shape, "ridge_k32_d4_d12", dtype=object)
        out[n > 12] = "ridge_k32_d16_d24"
        out[n > 24] = "ridge_k32_d28_up"
        return out
    dmax = min(k, 32)
    d = np.maximum(4, 4 * ((n + 3) // 4))
    names = np.array(["ridge_k%d_d%d" % (k, x) for x in range(0, 33)], dtype=object)
    out = names[np.minimum(d, 32)]
    out[n > dmax] = "ridge_k%d_primal" % k
    return out


def recorded_traffic(kernel, choice):
    """HBM bytes per launch of `kernel` in its chosen variant from the committed rocprofv3
    counter summary, or None when the summary covers another kernel or variant, or the kernel's
    sources changed since."""
    import hashlib
    path = os.path.join(HERE, "profiles", "ridge_foldin_1M_k32.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
    if not rec or rec.get("kernel") != kernel:
        return None
    by_choice = rec.get("traffic_by_choice", {})
    if str(choice) not in by_choice and rec.get("choice") != choice:
        return None
    h = hashlib.sha1()
    for f in rec["sources"]:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["sources_sha1"]:
        return None
    return by_choice.get(str(choice), rec["traffic_bytes_per_launch"])


def surrogate_leg(args, ctx, dV, drp, dcol, dval, m, steps, warmup, log, als_ms):
    """Surrogate fold-in (MLP + ridge fallback on rows whose observed-entry RMS residual exceeds
    tau): train through open_mlp_train on the ALS fold-ins of 2M new draws, then time
    surrogate+fallback on the benchmark rows, beside the same with the untrained network (same
    seeded initial weights), which falls back almost everywhere, and the plain ALS fold-in."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    c = synth.CONFIGS["surrogate"]
    grid = synth.grid_of("surrogate")
    n, k, lam, wt, tau = grid.n, c["k"], c["lam"], c["weighted"], c["tau"]
    dev = dV.device
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    t0 = time.time()
    tr = synth.draw_rows(c["cfg_id"], grid, c["m_train"], c["counts"], seed=c["train_seed"])
    trp, tcol, tval = to(tr.row_ptr), to(tr.col), to(tr.val)
    target = native.open_foldin(ctx, dV, trp, tcol, tval, lam, wt)
    torch.cuda.synchronize()
    log("surrogate: %d training rows and their ALS targets in %.1f s" % (tr.m, time.time() - t0))

    net = native.Surrogate(ctx, n, k, c["hidden"], seed=1)
    untrained = native.Surrogate(ctx, n, k, c["hidden"], seed=1)
    B, E = c["batch"], int(args.surrogate_epochs)
    torch.cuda.synchronize()
    t0 = time.time()
    hist = net.train(trp, tcol, tval, target, B, c["lr"], E, seed=7)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    n_steps = E * (tr.m // B)
    log("surrogate: %d epochs (%d Adam steps) in %.2f s, %.3f ms per step; epoch losses %s"
        % (E, n_steps, train_s, 1e3 * train_s / max(n_steps, 1), np.array2string(hist, precision=3)))
    del trp, tcol, tval, target

    U = torch.empty((m, k), dtype=torch.float32, device=dev)
    used = torch.empty(m, dtype=torch.uint8, device=dev)
    rho = torch.empty(m, dtype=torch.float32, device=dev)

    def timed(model):
        for _ in range(warmup):
            model.foldin(dV, drp, dcol, dval, tau, lam, wt, U_out=U, used_fallback=used, count=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            model.foldin(dV, drp, dcol, dval, tau, lam, wt, U_out=U, used_fallback=used, count=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        _, nf = model.foldin(dV, drp, dcol, dval, tau, lam, wt, U_out=U, used_fallback=used, rho=rho)
        return ms, nf

    ms0, nf0 = timed(untrained)
    ms, nf = timed(net)
    # the floor of any network that reproduces the ALS fold-in: rows whose own ALS residual is above tau
    Ua = native.open_foldin(ctx, dV, drp, dcol, dval, lam, wt)
    ra = native.open_residual(ctx, drp, dcol, dval, Ua, dV)
    als_above = float((ra > tau).float().mean().item())
    del Ua, ra
    ctx.profile(True)
    net.foldin(dV, drp, dcol, dval, tau, lam, wt, U_out=U, used_fallback=used, count=False)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    infer_ms = prof["mlp_infer"][0] if "mlp_infer" in prof else None
    flops = (2.0 * 256 * 2 * float(drp[-1].item()) + m * 2.0 * (256 * 256 + 256 * k))
    out = {
        "workload": "surrogate fold-in + ridge fallback: the %d benchmark rows, network %d-%d-%d-%d trained "
                    "%d epochs on %d ALS fold-ins, tau %g, plain lambda %g" % (m, 2 * n, c["hidden"], c["hidden"], k,
                                                                          E, tr.m, tau, lam),
        "rows_per_s": m / (ms * 1e-3), "ms_per_step": ms, "fallback_fraction": nf / m,
        "untrained_rows_per_s": m / (ms0 * 1e-3), "untrained_fallback_fraction": nf0 / m,
        "als_rows_per_s": m / (als_ms * 1e-3), "als_residual_above_tau_fraction": als_above,
        "train_steps": n_steps, "train_epochs": E, "train_rows": tr.m, "batch": B,
        "train_seconds": round(train_s, 3), "train_ms_per_step": round(1e3 * train_s / max(n_steps, 1), 4),
        "epoch_loss": [float(x) for x in hist], "tau": tau,
        "network": "%d-%d-%d-%d bf16 weights, fp32 accumulate" % (2 * n, c["hidden"], c["hidden"], k),
    }
    if infer_ms:
        tf = flops / (infer_ms * 1e-3) / 1e12
        out["infer_roofline"] = {"kernel": "mlp_infer", "kernel_ms": round(infer_ms, 4), "bound": "mfma",
                                 "achieved": round(tf, 2), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(tf / PEAK_BF16_TFLOPS, 4), "algorithmic_flops": flops}
    untrained.close()
    net.close()
    return out, U


def large_leg(args, ctx, steps, warmup, log):
    """The large grid: 2M apps x 1920 settings (48 x 40 caps), ~2 % observed (truncated Zipf on
    [3, 1920]), rank 64.  ALS-WR fit of 10 sweeps from the generator's initial factors (time per
    sweep), then the fused predict + Algorithm 2 selection over all 1920 settings of every app
    with the fitted factors, then the surrogate 3840-256-256-64 trained at batch 16384 on the
    fold-ins of the fitted apps against the fitted setting factors, used with the ridge fallback
    on 200k new apps."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    c = synth.CONFIGS["large"]
    grid = synth.grid_of("large")
    k, lam, m = c["k"], c["lam"], c["m"]
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    t0 = time.time()
    rows = synth.draw_rows(c["cfg_id"], grid, m, c["counts"], seed=0)
    U0, V0 = synth.init_factors(c["cfg_id"], m, grid.n, k)
    drp, dcol, dval = to(rows.row_ptr), to(rows.col), to(rows.val)
    log("large: %d apps x %d settings, %d observed, generated in %.1f s" % (m, grid.n, rows.nnz, time.time() - t0))
    out = {}

    # ---- fit
    dU, dV = to(U0), to(V0)

    def timed_fit(sweeps):
        dU.copy_(to(U0))
        dV.copy_(to(V0))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        native.open_fit(ctx, drp, dcol, dval, dU, dV, lam, sweeps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    timed_fit(1)  # warm-up (workspaces, code)
    t1 = timed_fit(1)
    S = c["sweeps"]
    tS = timed_fit(S)
    ms = (tS - t1) / (S - 1)
    obj = native.open_objective(ctx, drp, dcol, dval, dU, dV, lam)
    ccount = np.bincount(rows.col, minlength=grid.n)
    flops = float(row_flops(rows.counts(), k).sum() + row_flops(ccount, k).sum())
    tf = flops / (ms * 1e-3) / 1e12
    out["fit"] = {"workload": "ALS-WR fit: %d apps x %d settings (48 x 40 caps), %d observed (truncated Zipf 1.6931 on "
                              "[3, 1920]), rank %d, weighted lambda %g, %d sweeps" % (m, grid.n, rows.nnz, k, lam, S),
                  "ms_per_sweep": ms, "ms_total_%d_sweeps" % S: tS, "setup_ms_per_call": t1 - ms,
                  "objective_after": obj,
                  "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(tf / PEAK_FP32_TFLOPS, 4), "algorithmic_flops": flops}}
    log("large fit: %.3f ms per sweep (%.1f TFLOP/s), objective %.6g" % (ms, tf, obj))

    # ---- predict + Algorithm 2 with the fitted factors
    cc, cg = to(grid.cpu_w.astype(np.float32)), to(grid.gpu_w.astype(np.float32))
    bi = torch.empty(m, dtype=torch.int32, device=dev)
    bs = torch.empty(m, dtype=torch.float32, device=dev)
    run = lambda: native.open_predict(ctx, dU, dV, cc, cg, grid.base, c["gamma"], best_idx=bi, best_saving=bs)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / steps
    pflops = 2.0 * k * grid.n * m
    pbytes = (4.0 * k + 8.0) * m
    ptf = pflops / (pms * 1e-3) / 1e12
    out["predict_select"] = {
        "workload": "predict + Alg. 2 selection with the fitted factors: %d apps x %d settings, rank %d, gamma %g"
                    % (m, grid.n, k, c["gamma"]),
        "rows_per_s": m / (pms * 1e-3), "ms_per_step": pms,
        "chosen_not_baseline_fraction": float((bi != grid.base).float().mean().item()),
        "mean_saving": float(bs.mean().item()),
        "roofline": {"bound": "mfma", "achieved": round(ptf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ptf / PEAK_FP32_TFLOPS, 4), "algorithmic_flops": pflops,
                     "algorithmic_bytes": pbytes, "hbm_gbs": round(pbytes / (pms * 1e-3) / 1e9, 1)}}
    log("large predict+select %.3e rows/s, %.1f TFLOP/s" % (m / (pms * 1e-3), ptf))
    del bi, bs

    # ---- surrogate at rank 64, batch 16384, with the ridge fallback
    if not args.no_surrogate:
        wt, tau, B, E = False, 0.02, c["batch"], int(args.surrogate_epochs)
        target = native.open_foldin(ctx, dV, drp, dcol, dval, lam, wt)
        net = native.Surrogate(ctx, grid.n, k, c["hidden"], seed=1)
        untrained = native.Surrogate(ctx, grid.n, k, c["hidden"], seed=1)
        torch.cuda.synchronize()
        t0 = time.time()
        hist = net.train(drp, dcol, dval, target, B, 1e-3, E, seed=7)
        torch.cuda.synchronize()
        train_s = time.time() - t0
        nsteps = E * (m // B)
        log("large surrogate: %d epochs (%d steps at batch %d) in %.2f s; epoch losses %s"
            % (E, nsteps, B, train_s, np.array2string(hist, precision=3)))
        del target
        new = synth.draw_rows(c["cfg_id"], grid, 200_000, c["counts"], seed=1)
        nrp, ncol, nval = to(new.row_ptr), to(new.col), to(new.val)
        Un = torch.empty((new.m, k), dtype=torch.float32, device=dev)

        def timed(fn):
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        ms_als = timed(lambda: native.open_foldin(ctx, dV, nrp, ncol, nval, lam, wt, U_out=Un))
        Ua = Un.clone()
        als_above = float((native.open_residual(ctx, nrp, ncol, nval, Ua, dV) > tau).float().mean().item())
        ms_u = timed(lambda: untrained.foldin(dV, nrp, ncol, nval, tau, lam, wt, U_out=Un, count=False))
        _, nf_u = untrained.foldin(dV, nrp, ncol, nval, tau, lam, wt, U_out=Un)
        ms_t = timed(lambda: net.foldin(dV, nrp, ncol, nval, tau, lam, wt, U_out=Un, count=False))
        _, nf_t = net.foldin(dV, nrp, ncol, nval, tau, lam, wt, U_out=Un)
        # RMSE against the noiseless truth on unobserved settings of 5,000 new apps
        ev = np.arange(0, new.m, 40)
        T = synth.truth_dense(new.apps.take(ev), grid)
        obs = np.zeros_like(T, dtype=bool)
        for j, i in enumerate(ev):
            obs[j, new.col[new.row_ptr[i]:new.row_ptr[i + 1]]] = True
        Vd = dV.cpu().numpy().astype(np.float64)
        idx = torch.from_numpy(ev).to(dev)
        rm = lambda U: float(np.sqrt((((U[idx].cpu().numpy().astype(np.float64) @ Vd.T) - T)[~obs] ** 2).mean()))
        r_s, r_a = rm(Un), rm(Ua)
        out["surrogate"] = {
            "workload": "surrogate fold-in + ridge fallback on 200000 new apps of the large grid: network %d-%d-%d-%d "
                        "trained %d epochs at batch %d on the fold-ins of the %d fitted apps, tau %g, plain lambda %g"
                        % (2 * grid.n, c["hidden"], c["hidden"], k, E, B, m, tau, lam),
            "rows_per_s": new.m / (ms_t * 1e-3), "fallback_fraction": nf_t / new.m,
            "untrained_rows_per_s": new.m / (ms_u * 1e-3), "untrained_fallback_fraction": nf_u / new.m,
            "als_rows_per_s": new.m / (ms_als * 1e-3), "als_residual_above_tau_fraction": als_above,
            "train_seconds": round(train_s, 3),
            "train_ms_per_step": round(1e3 * train_s / max(nsteps, 1), 4), "epoch_loss": [float(x) for x in hist],
            "rmse": r_s, "rmse_gpu_als": r_a, "rmse_gap_vs_gpu_als": abs(r_s - r_a)}
        log("large surrogate+fallback %.3e rows/s (fallback %.3f), untrained %.3e (fallback %.3f), ALS %.3e; "
            "RMSE %.5f vs ALS %.5f" % (new.m / (ms_t * 1e-3), nf_t / new.m, new.m / (ms_u * 1e-3), nf_u / new.m,
                                       new.m / (ms_als * 1e-3), r_s, r_a))
        net.close()
        untrained.close()
    return out


def phase_leg(ctx, steps, warmup, log):
    """Algorithm 1 (phase-transition detection) over 65,536 GPU power traces of 3000 readings
    (10 min at 0.2 s): traces per second and HBM bytes actually needed (4 B per reading up to
    each report, all readings of traces without one)."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    T, L = 65536, 3000
    t0 = time.time()
    P = torch.from_numpy(synth.power_traces(7, T, L, seed=0)).cuda()
    log("phase: %d traces x %d readings in %.1f s" % (T, L, time.time() - t0))
    out = torch.empty(T, dtype=torch.int64, device=P.device)
    for _ in range(warmup):
        native.open_phase_detect(ctx, P, 60.0, 25, first_index=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        native.open_phase_detect(ctx, P, 60.0, 25, first_index=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    f = out.cpu().numpy()
    byts = float(np.where(f >= 0, f + 1, L).sum() * 4)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": "Alg. 1 phase detection: %d power traces x %d readings, window 25, 60 W" % (T, L),
            "traces_per_s": T / (ms * 1e-3), "ms_per_step": ms, "detected_fraction": float((f >= 0).mean()),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": byts}}


def predictor_leg(ctx, rows, grid, steps, warmup, log):
    """Offline performance predictor (7 -> 64 -> 64 -> 1) over every profiled run of the fold-in
    workload (one feature vector per observed entry): runs per second.  Algorithmic work per
    run: 2 (7*64 + 64*64 + 64) = 9216 flop and 32 B of HBM (28 B of features, 4 B out); the
    kernel issues twice the layer products on BF16 MFMA (two-part activations)."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    t0 = time.time()
    X = torch.from_numpy(synth.run_features(3, grid, rows.col)).cuda()
    p = {k: torch.from_numpy(v).cuda() for k, v in synth.predictor_params(3, grid).items()}
    n = X.shape[0]
    log("predictor: %d runs in %.1f s" % (n, time.time() - t0))
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    for _ in range(warmup):
        native.open_perf_predict(ctx, X, p, y=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        native.open_perf_predict(ctx, X, p, y=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops, byts = 9216.0 * n, 32.0 * n
    tf = flops / (ms * 1e-3) / 1e12
    gbs = byts / (ms * 1e-3) / 1e9
    return {"workload": "offline predictor 7-64-64-1 (ReLU) over the %d profiled runs of the fold-in workload" % n,
            "runs_per_s": n / (ms * 1e-3), "ms_per_step": ms,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": byts,
                         "bf16_mfma_tflops": round(tf, 2), "bf16_mfma_frac": round(tf / PEAK_BF16_TFLOPS, 4)}}


def ncf_leg(ctx, steps, warmup, log):
    """NCF (Section III-B.1 model): trained on the GPU (open_ncf_train, 20 epochs, 8 applications
    x 480 settings per batch, Adam 1e-3) on the dense offline matrix of the 4096 reference apps
    (the same noiseless matrix whose truncated SVD gives the ALS setting factors); then the
    NCF fold-in (embedding learned by 30 gradient steps per new app, products on FP32 MFMA)
    of 65,536 new apps with 4-24 observed settings each: apps per second, and the RMSE of NCF
    and of the plain-lambda ALS fold-in against the noiseless truth on unobserved settings of
    20,000 of them.  Algorithmic work per observed entry and step of the fold-in: forward
    2 (32*64 + 64*64 + 64) flop, backward 2 (64 + 64*64) flop, plus 2*32*64 flop per app and
    step for the embedding layer both ways."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    c = synth.NCF
    grid = synth.grid_of("foldin")
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # offline training
    m_off = 4096
    R = synth.truth_dense(synth.draw_apps(synth.rng(3, synth.S_REF, 0), m_off), grid).astype(np.float32)
    p0 = synth.ncf_params(3, grid.n)
    S0 = p0.pop("S")
    flat = to(native.ncf_pack(np.zeros((m_off, 32), np.float32), S0, p0))
    dR = to(R)
    G, E_train = 8, 20
    torch.cuda.synchronize()
    t0 = time.time()
    hist = native.open_ncf_train(ctx, dR, flat, G, 1e-3, E_train, seed=1)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    nsteps = E_train * (m_off // G)
    log("NCF training: %d epochs (%d steps of %d entries) in %.2f s, epoch losses %s"
        % (E_train, nsteps, G * grid.n, train_s, np.array2string(hist, precision=5)))
    _, S, net = native.ncf_unpack(flat, m_off, grid.n)
    # fold-in of new apps
    m = 65_536
    rows = synth.draw_rows(3, grid, m, ("uniform", 4, 24), seed=0)
    drp, dcol, dval = to(rows.row_ptr), to(rows.col), to(rows.val)
    E = torch.empty((m, 32), dtype=torch.float32, device=dev)
    L = torch.empty(m, dtype=torch.float32, device=dev)
    reps = max(1, steps // 4)
    for _ in range(max(1, warmup // 2)):
        native.open_ncf_foldin(ctx, S, net, drp, dcol, dval, c["steps"], c["eta"], c["mu"], E_out=E, loss_out=L)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        native.open_ncf_foldin(ctx, S, net, drp, dcol, dval, c["steps"], c["eta"], c["mu"], E_out=E, loss_out=L)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nnz = float(rows.nnz)
    flops = c["steps"] * (nnz * 2 * (32 * 64 + 64 * 64 + 64 + 64 + 64 * 64) + m * 2 * 2 * 32 * 64)
    tf = flops / (ms * 1e-3) / 1e12
    # accuracy of NCF and ALS on 20,000 of the new apps (unobserved settings, noiseless truth)
    ev = np.arange(20_000)
    T = synth.truth_dense(rows.apps.take(ev), grid)
    obs = np.zeros_like(T, dtype=bool)
    for i in ev:
        obs[i, rows.col[rows.row_ptr[i]:rows.row_ptr[i + 1]]] = True
    with torch.no_grad():
        Ee = E[:len(ev)].double()
        X1 = torch.cat([Ee[:, None, :].expand(-1, grid.n, -1), S.double()[None].expand(len(ev), -1, -1)], dim=2)
        selu = lambda z: 1.0507009873554805 * torch.where(z > 0, z, 1.6732632423543772 * torch.expm1(torch.clamp(z, max=0)))
        h1 = selu(X1 @ net["W1"].double().T + net["b1"].double())
        h2 = selu(h1 @ net["W2"].double().T + net["b2"].double())
        P_ncf = (h2 @ net["w3"].double() + net["b3"].double()[0]).cpu().numpy()
    V = synth.setting_factors(3, grid, 32)
    cf = synth.CONFIGS["foldin"]
    Ua = native.open_foldin(ctx, to(V), drp, dcol, dval, cf["lam"], cf["weighted"])[:len(ev)].cpu().numpy()
    P_als = Ua.astype(np.float64) @ V.astype(np.float64).T
    rmse = lambda P: float(np.sqrt(((P - T)[~obs] ** 2).mean()))
    return {"workload": "NCF: trained %d epochs on the 4096 x 480 reference matrix (%.2f s, %.3f ms per step of %d "
                        "entries); fold-in of %d new apps x 480 settings, 4-24 observed, embedding 32, SELU 64-64, "
                        "%d gradient steps" % (E_train, train_s, 1e3 * train_s / nsteps, G * grid.n, m, c["steps"]),
            "apps_per_s": m / (ms * 1e-3), "ms_per_call": ms, "mean_final_loss": float(L.mean().item()),
            "train_epoch_loss": [float(x) for x in hist], "train_seconds": round(train_s, 3),
            "rmse_ncf": rmse(P_ncf), "rmse_als_foldin": rmse(P_als),
            "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / PEAK_FP32_TFLOPS, 4), "algorithmic_flops": flops}}


def refit_leg(ctx, state, log):
    """Warm-started refit: 50k new apps (4-24 observed each) arrive at the fitted 200k x 480
    matrix; fold-in alone vs fold-in + 2 ALS sweeps on the union, timed, with the RMSE of both
    against the noiseless truth on the new apps' unobserved settings."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    c, grid, rows, dU, dV = state
    k, lam = c["k"], c["lam"]
    new = synth.draw_rows(c["cfg_id"], grid, 50_000, ("uniform", 4, 24), seed=1)
    rp = np.concatenate([rows.row_ptr, rows.row_ptr[-1] + new.row_ptr[1:]])
    col = np.concatenate([rows.col, new.col])
    val = np.concatenate([rows.val, new.val])
    dev = dU.device
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    drp, dcol, dval = to(rp), to(col), to(val)
    m_old, m = rows.m, rows.m + new.m
    U_f = torch.cat([dU, torch.zeros((new.m, k), dtype=torch.float32, device=dev)])
    V_f = dV.clone()
    native.open_refit(ctx, m_old, drp, dcol, dval, U_f, V_f, lam, 0)  # fold-in only
    U_r, V_r = U_f.clone(), dV.clone()
    U_r[m_old:] = 0
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    native.open_refit(ctx, m_old, drp, dcol, dval, U_r, V_r, lam, 2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ev = np.sort(np.random.default_rng(5).choice(new.m, size=10_000, replace=False))
    T = synth.truth_dense(new.apps.take(ev), grid)
    obs = np.zeros_like(T, dtype=bool)
    for j, i in enumerate(ev):
        obs[j, new.col[new.row_ptr[i]:new.row_ptr[i + 1]]] = True
    idx = torch.from_numpy(ev + m_old).to(dev)

    def rmse(U, V):
        P = (U[idx].double() @ V.double().T).cpu().numpy()
        return float(np.sqrt(((P - T)[~obs] ** 2).mean()))

    r_f, r_r = rmse(U_f, V_f), rmse(U_r, V_r)
    log("refit: 2 sweeps on %d rows in %.2f ms; new-app RMSE fold-in %.5f, refit %.5f" % (m, ms, r_f, r_r))
    return {"workload": "warm refit: %d offline + %d new apps x %d settings, rank %d, 2 sweeps" %
                        (m_old, new.m, grid.n, k),
            "ms": ms, "rmse_new_foldin": r_f, "rmse_new_refit": r_r, "drift": r_f - r_r}


def fit_leg(args, ctx, log, name="fit"):
    """ALS-WR fit on 200k apps x 480 settings, rank 32, weighted lambda 0.05, observed counts
    truncated Zipf on [3, 480]: exponent 1.2 ("fit", 12.7M observed entries) or 1.6824 ("fit_d5",
    5 % density): time per sweep (rows, then columns), objective after the timed sweeps."""
    import numpy as np
    import torch

    from paper_2508_07605_amd import native, synth

    c = synth.CONFIGS[name]
    grid = synth.grid_of(name)
    k, lam = c["k"], c["lam"]
    t0 = time.time()
    rows = synth.draw_rows(c["cfg_id"], grid, c["m"], c["counts"], seed=0)
    U0, V0 = synth.init_factors(c["cfg_id"], rows.m, grid.n, k)
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    drp, dcol, dval = to(rows.row_ptr), to(rows.col), to(rows.val)
    dU, dV = to(U0), to(V0)
    log("%s: %d rows, %d nnz in %.1f s" % (name, rows.m, rows.nnz, time.time() - t0))
    native.open_fit(ctx, drp, dcol, dval, dU, dV, lam, 1)  # warm-up sweep (workspaces, code)
    torch.cuda.synchronize()
    S = args.fit_sweeps

    def timed_fit(sweeps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        native.open_fit(ctx, drp, dcol, dval, dU, dV, lam, sweeps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t1 = timed_fit(1)
    tS = timed_fit(S + 1)
    ms = (tS - t1) / S          # one more sweep, setup excluded
    setup_ms = t1 - ms          # column view, bucketings, temporaries of one call
    ctx.profile(True)
    native.open_fit(ctx, drp, dcol, dval, dU, dV, lam, 1)
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    log("%s: kernels (one call, one sweep) %s" % (name, json.dumps({n: round(t, 4) for n, (t, c) in prof.items()})))
    obj = native.open_objective(ctx, drp, dcol, dval, dU, dV, lam)
    ccount = np.bincount(rows.col, minlength=grid.n)
    flops = float(row_flops(rows.counts(), k).sum() + row_flops(ccount, k).sum())
    tf = flops / (ms * 1e-3) / 1e12
    state = (c, grid, rows, dU, dV)
    _, zexp, zlo, zhi = c["counts"]
    return state, {"workload": "ALS-WR fit: %d apps x %d settings, Zipf(%g) counts on [%d, %d], %d nnz (density %.1f %%), "
                        "rank %d, weighted lambda %g" % (rows.m, grid.n, zexp, zlo, zhi, rows.nnz,
                                                         100.0 * rows.nnz / (rows.m * grid.n), k, lam),
            "ms_per_sweep": ms, "setup_ms_per_call": setup_ms, "sweeps_timed": S, "objective_after": obj,
            "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / PEAK_FP32_TFLOPS, 4), "algorithmic_flops": flops}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=None, help="override the 1,000,000 new rows")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle work for the CPU baseline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 256 MiB device copy (reference kernel for HBM counter scaling)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default kernel variants")
    ap.add_argument("--graph", action="store_true", help="time the pass as one HIP graph replay instead of "
                                                          "kernel-by-kernel launches")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate (MLP + fallback) leg")
    ap.add_argument("--no-large", action="store_true", help="skip the large-grid leg (fit, predict + selection, "
                                                              "rank-64 surrogate)")
    ap.add_argument("--no-fit", action="store_true", help="skip the ALS fit leg")
    ap.add_argument("--no-phase", action="store_true", help="skip the Alg. 1 phase-detection leg")
    ap.add_argument("--no-predictor", action="store_true", help="skip the offline performance predictor leg")
    ap.add_argument("--no-ncf", action="store_true", help="skip the NCF fold-in leg")
    ap.add_argument("--fit-sweeps", type=int, default=3, help="timed ALS sweeps in the fit leg")
    ap.add_argument("--surrogate-epochs", type=int, default=10,
                    help="training epochs over the 2M ALS fold-in targets (batch 4096, Adam 1e-3)")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of autotuned kernel variants")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: only one GPU is measured; the row-parallel legs would shard rows across GPUs "
              "with no exchange. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2508_07605_amd import autotune, native, synth

    cfg = synth.CONFIGS["foldin"]
    k, lam, wt = cfg["k"], cfg["lam"], cfg["weighted"]
    m = args.rows or cfg["m"]
    grid = synth.grid_of("foldin")
    t0 = time.time()
    V = synth.setting_factors(cfg["cfg_id"], grid, k)
    rows = synth.draw_rows(cfg["cfg_id"], grid, m, cfg["counts"], seed=0)
    print("bench: generated %d rows (%d nnz) in %.1f s" % (m, rows.nnz, time.time() - t0), file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dV, drp, dcol, dval = to(V), to(rows.row_ptr), to(rows.col), to(rows.val)
    dU = torch.empty((m, k), dtype=torch.float32, device=dev)
    dst = torch.empty(m, dtype=torch.int32, device=dev)
    ctx = native.Context(0)

    def step_eager():
        native.open_foldin(ctx, dV, drp, dcol, dval, lam, wt, U_out=dU, row_status=dst)

    def step_graph():
        native.open_foldin_graph(ctx, dV, drp, dcol, dval, lam, wt, U_out=dU, row_status=dst)

    step = step_graph if args.graph else step_eager

    if args.copy_calib:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # setup, outside the timed region: pick the kernel variant of each size class on this batch
    tune_table = None
    if not args.no_autotune:
        t0 = time.time()
        _, tune_table = autotune.tune(ctx, dV, drp, dcol, dval, lam, wt, reps=3, path=args.tune_cache)
        print("bench: autotune %.1f s, variants %s, ms %s" % (time.time() - t0, ctx.tune_get(k), tune_table),
              file=sys.stderr, flush=True)
    variants = dict(zip([g for g, _ in native.open_tune_info(k)], ctx.tune_get(k)))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = m / (ms * 1e-3)
    print("bench: %d steps, %.3f ms/step, %.3e rows/s" % (args.steps, ms, value), file=sys.stderr, flush=True)
    st = dst.cpu().numpy()
    assert (st == 0).all(), "row status not ok: %s" % np.bincount(st)

    # live per-kernel timing (HIP events around each launch, on the library's stream)
    # the other launch mode of the same pass
    other = step_eager if args.graph else step_graph
    for _ in range(args.warmup):
        other()
    torch.cuda.synchronize()
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev2.record()
    for _ in range(args.steps):
        other()
    ev3.record()
    torch.cuda.synchronize()
    other_ms = ev2.elapsed_time(ev3) / args.steps
    # per-kernel timing, kernel by kernel (a graph replay has no per-kernel events)
    ctx.profile(True)
    for _ in range(args.profile_steps):
        step_eager()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    counts = rows.counts()
    tiers = kernel_of_counts(counts, k, variants.get("ridge_k%d_launch" % k, 1))
    flops = row_flops(counts, k)
    kernels = {}
    for name, (tot, launches) in prof.items():
        avg_ms = tot / launches
        kernels[name] = avg_ms
    ridge = {n: t for n, t in kernels.items() if n.startswith("ridge_")}
    dom = max(ridge, key=ridge.get)
    sel = tiers == dom
    dom_flops = float(flops[sel].sum())
    dom_rows = int(sel.sum())
    dom_bytes = float((8 * counts[sel] + 8 + 4 * k).sum())
    dom_ms = ridge[dom]
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    roofline = {
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": recorded_traffic(dom, variants.get(dom, -1)),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "kernel": dom, "kernel_ms": round(dom_ms, 4), "kernel_rows": dom_rows,
        "algorithmic_flops": dom_flops, "algorithmic_bytes": dom_bytes,
        "hbm_gbs": round(dom_bytes / (dom_ms * 1e-3) / 1e9, 1),
    }
    all_flops = float(flops.sum())
    pass_tflops = all_flops / (ms * 1e-3) / 1e12
    print("bench: kernels %s" % json.dumps({n: round(t, 4) for n, t in kernels.items()}), file=sys.stderr, flush=True)

    out = {
        "metric": "fold-in rows/sec at rank 32 (ALS vs MLP) at equal RMSE vs FP64 oracle",
        "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched ALS fold-in: %d new apps x 480 settings (24 CPU x 20 GPU caps), "
                               "4-24 observed per app, rank 32, plain lambda 0.05, fixed float32 setting factors"
                               % m, "rows": m, "settings": grid.n, "rank": k, "nnz": rows.nnz,
                   "parallelism": "single GPU", "kernel_variants": variants},
        "pass_tflops": round(pass_tflops, 3),
        "launch": "one HIP graph replay per pass" if args.graph else "kernel by kernel",
        ("eager_ms_per_step" if args.graph else "graph_ms_per_step"): other_ms,
        "roofline": roofline,
    }

    log = lambda msg: print("bench: " + msg, file=sys.stderr, flush=True)
    if not args.no_large:
        out["large"] = large_leg(args, ctx, args.steps, args.warmup, log)
    if not args.no_phase:
        out["phase_detect"] = phase_leg(ctx, args.steps, args.warmup, log)
        log("phase detection %.3e traces/s, %.0f GB/s" % (out["phase_detect"]["traces_per_s"],
                                                           out["phase_detect"]["roofline"]["achieved"]))
    if not args.no_predictor:
        out["perf_predictor"] = predictor_leg(ctx, rows, grid, args.steps, args.warmup, log)
        log("offline predictor %.3e runs/s, %.0f GB/s, %.1f TFLOP/s" % (
            out["perf_predictor"]["runs_per_s"], out["perf_predictor"]["roofline"]["achieved"],
            out["perf_predictor"]["roofline"]["bf16_mfma_tflops"]))
    if not args.no_ncf:
        out["ncf_foldin"] = ncf_leg(ctx, args.steps, args.warmup, log)
        log("NCF fold-in %.3e apps/s (%.3f ms), %.1f TFLOP/s; RMSE NCF %.5f vs ALS fold-in %.5f" % (
            out["ncf_foldin"]["apps_per_s"], out["ncf_foldin"]["ms_per_call"],
            out["ncf_foldin"]["roofline"]["achieved"], out["ncf_foldin"]["rmse_ncf"],
            out["ncf_foldin"]["rmse_als_foldin"]))
    if not args.no_fit:
        fit_state, out["fit"] = fit_leg(args, ctx, log)
        out["refit"] = refit_leg(ctx, fit_state, log)
        del fit_state
        _, out["fit_d5"] = fit_leg(args, ctx, log, "fit_d5")
        log("fit %.3f ms/sweep, %.1f TFLOP/s; fit_d5 %.3f ms/sweep, %.1f TFLOP/s"
            % (out["fit"]["ms_per_sweep"], out["fit"]["roofline"]["achieved"], out["fit_d5"]["ms_per_sweep"],
               out["fit_d5"]["roofline"]["achieved"]))
    U_sur = None
    if not args.no_surrogate:
        log = lambda msg: print("bench: " + msg, file=sys.stderr, flush=True)
        sur, U_sur = surrogate_leg(args, ctx, dV, drp, dcol, dval, m, args.steps, args.warmup, log, ms)
        out["surrogate"] = sur
        log("surrogate+fallback %.3e rows/s (fallback %.3f), untrained %.3e rows/s (fallback %.3f)"
            % (sur["rows_per_s"], sur["fallback_fraction"], sur["untrained_rows_per_s"],
               sur["untrained_fallback_fraction"]))

    # accuracy: both fold-ins against the noiseless truth on unobserved settings of sampled rows
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        rs = np.random.default_rng(2025)
        probe = np.sort(rs.choice(m, size=min(m, 20_000), replace=False))
        t1 = time.perf_counter()
        oracle.ridge_subset(probe, rows.row_ptr, rows.col, rows.val, V, lam, wt)
        per_row = (time.perf_counter() - t1) / len(probe)
        ns = int(min(m, max(len(probe), args.cpu_seconds / max(per_row, 1e-9))))
        sample = np.sort(rs.choice(m, size=ns, replace=False))
        # the sample solved repeatedly until about cpu_seconds of work (the whole workload can
        # take less than that on the host's cores)
        reps, cpu_s = 0, 0.0
        while reps == 0 or cpu_s < args.cpu_seconds:
            t1 = time.perf_counter()
            Uref, st_ref = oracle.ridge_subset(sample, rows.row_ptr, rows.col, rows.val, V, lam, wt)
            cpu_s += time.perf_counter() - t1
            reps += 1
        # one thread on a smaller sample, about a quarter of that time
        one = sample[:max(1, min(ns, int(args.cpu_seconds / 4 / max(per_row * threads, 1e-9))))]
        oracle.set_threads(1)
        t1 = time.perf_counter()
        oracle.ridge_subset(one, rows.row_ptr, rows.col, rows.val, V, lam, wt)
        cpu1_s = time.perf_counter() - t1
        oracle.set_threads(threads)
        cpu_model = None
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        out["cpu_baseline"] = {"value": reps * ns / cpu_s, "unit": "rows/s", "cores": threads, "kind": "oracle",
                               "sample": "%d of the %d rows (seeded), FP64 primal ridge solves, solved %d times "
                                         "in %.1f s" % (ns, m, reps, cpu_s),
                               "single_thread": {"value": len(one) / cpu1_s, "unit": "rows/s", "cores": 1,
                                                 "sample": "the first %d rows of that sample, %.1f s"
                                                           % (len(one), cpu1_s)},
                               "cpu_model": cpu_model, "host_cpus": os.cpu_count()}
        ev = sample[:20_000]
        Ug = dU[torch.from_numpy(ev).to(dev)].cpu().numpy().astype(np.float64)
        Uo = Uref[:len(ev)]
        T = synth.truth_dense(rows.apps.take(ev), grid)
        obs = np.zeros_like(T, dtype=bool)
        sub_rp = rows.row_ptr
        for j, i in enumerate(ev):
            obs[j, rows.col[sub_rp[i]:sub_rp[i + 1]]] = True
        Vd = V.astype(np.float64)
        rmse_g = float(np.sqrt((((Ug @ Vd.T) - T)[~obs] ** 2).mean()))
        rmse_o = float(np.sqrt((((Uo @ Vd.T) - T)[~obs] ** 2).mean()))
        # the other lambda convention (lambda n_i), for the reading of the fold-in's regulariser
        Uw, _ = oracle.ridge_subset(ev, rows.row_ptr, rows.col, rows.val, V, lam, not wt)
        rmse_w = float(np.sqrt((((Uw @ Vd.T) - T)[~obs] ** 2).mean()))
        e = np.linalg.norm(Ug - Uo, axis=1) / np.linalg.norm(Uo, axis=1)
        if U_sur is not None:
            Us = U_sur[torch.from_numpy(ev).to(dev)].cpu().numpy().astype(np.float64)
            rmse_s = float(np.sqrt((((Us @ Vd.T) - T)[~obs] ** 2).mean()))
            out["surrogate"].update({"rmse": rmse_s, "rmse_gap_vs_oracle_als": abs(rmse_s - rmse_o),
                                     "pred_rmse_vs_oracle_als": float(np.sqrt(((((Us - Uo) @ Vd.T))[~obs] ** 2)
                                                                              .mean()))})
        out["accuracy"] = {"rows": len(ev), "rmse_gpu": rmse_g, "rmse_oracle": rmse_o,
                           "rmse_gap": abs(rmse_g - rmse_o), "max_rel_err_vs_oracle": float(e.max()),
                           ("rmse_oracle_weighted_lambda" if not wt else "rmse_oracle_plain_lambda"): rmse_w,
                           "accuracy_pct_1_minus_mape": float(100 * (1 - np.abs(((Ug @ Vd.T) - T)[~obs] /
                                                                               T[~obs]).mean()))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
