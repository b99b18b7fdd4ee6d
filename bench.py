"""Benchmark: damped Gauss-Newton steps/s of the medium CCF profile workload
on one MI355X, with the Gram kernel's roofline fraction and the CPU oracle
timed beside it.

One step = the whole hot path for one batch of collocation points: forward
jets, residual and validation max-norm, Jacobian (local sweeps + Hilbert
coupling GEMM), Gram of [J | r] (FP64 MFMA), bordered blocked Cholesky, back
substitution and the update of theta.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)
PEAK_INT8_TOPS = 5000.0  # MI355X dense int8 MFMA
PEAK_HBM_GBS = 8000.0    # MI355X HBM3E
METRIC = "Gauss-Newton steps/sec at fixed residual max-norm; Gram+Cholesky % FP64-MFMA peak"


def flops(P, m, n, mq):
    """Algorithmic flop counts of one step."""
    return {
        # lower triangle incl. diagonal of the (P+1)x(P+1) Gram of [J | r], 2 flops per MAC
        "gram": float(m) * (P + 1) * (P + 2),
        # Cholesky of the bordered (P+1) matrix
        "cholesky": (P + 1) ** 3 / 3.0,
        # Hilbert coupling GEMM N x M x P
        "coupling": 2.0 * n * mq * P,
    }


def gram_source_sha256():
    """sha256 over the Gram kernel's sources (k_dgemm.hip, then tile_loader.h)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("k_dgemm.hip", "tile_loader.h"):
        with open(os.path.join(ROOT, "paper_2509_14185_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def gram_traffic():
    """HBM bytes of one Gram (the product launch plus the launch that sums the
    split tiles) from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (profiles/gram_ccf_medium_pmc.txt, scaled by a plain copy of known size),
    or None if the GEMM source changed since."""
    path = os.path.join(ROOT, "profiles", "gram_ccf_medium_pmc.txt")
    try:
        kv = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l and not l.startswith("#"))
        if kv.get("kernel_source_sha256") != gram_source_sha256():
            return None
        return float(kv["gram_phase_hbm_traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def split_comparison(inp, theta0, mu, steps, target, fp64_elapsed):
    """Split-precision form (FP32 hi/lo Gram, FP64 residual/gradient/solve)
    from the same start theta0: steps/s over the same number of steps and the
    steps and time needed to reach the FP64 run's final validation max-norm
    (within 5%), capped at three times as many steps."""
    import torch

    from paper_2509_14185_amd import gn

    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                      precision="split32")
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    theta = torch.from_numpy(theta0.copy()).cuda()
    prob.step(theta.clone(), mu, stats=False)  # warm-up on a copy
    torch.cuda.synchronize()
    prob.profile_enable(True, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    final = prob.eval(theta)["max_abs_R_val"]
    # steps to reach the FP64 target (time = steps x measured step time)
    theta2 = torch.from_numpy(theta0.copy()).cuda()
    reached = None
    for k in range(1, 3 * steps + 1):
        st = prob.step(theta2, mu)
        if prob.eval(theta2)["max_abs_R_val"] <= 1.05 * target:
            reached = k
            break
    prob.close()
    return {
        "value": steps / el,
        "unit": "steps/s",
        "ms_per_step": 1e3 * el / steps,
        "gram_ms": phases["gram"] / nrec,
        "max_abs_R_val_final": final,
        "target_max_abs_R_val": target,
        "steps_to_target": reached,
        "time_to_target_s": None if reached is None else reached * el / steps,
        "fp64_steps_to_target": steps,
        "fp64_time_to_target_s": fp64_elapsed,
    }


def int8crt_comparison(inp, theta0, mu, steps, fp64_theta, fp64_final, gram_flops):
    """Gram from int8 matrix products by exact modular arithmetic (precision
    "int8crt"; residual, gradient, Cholesky and update FP64) over the same
    timed steps as the FP64 run from the same start theta0 (warm-up on a
    copy): steps/s, the Gram's time, its FP64-equivalent rate and its int8
    rate against the int8 MFMA peak, and how far the final iterate is from the
    FP64 run's."""
    import torch

    from paper_2509_14185_amd import gn

    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                      precision="int8crt")
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    theta = torch.from_numpy(theta0.copy()).cuda()
    prob.step(theta.clone(), mu, stats=False)  # warm-up on a copy
    torch.cuda.synchronize()
    prob.profile_enable(True, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    final = prob.eval(theta)["max_abs_R_val"]
    m = prob.m
    prob.close()
    P = len(inp["theta0"])  # the modular Gram covers the parameter columns; g and r^T r are FP64
    bits, mods = gn.int8_crt_params(m)
    ppad = -(-P // 256) * 256
    kpad = -(-m // 128) * 128
    tiles = ppad // 256
    int8_ops = len(mods) * tiles * (tiles + 1) // 2 * 256 * 256 * kpad * 2
    t_gram = phases["gram"] / nrec * 1e-3
    return {
        "value": steps / el,
        "unit": "steps/s",
        "ms_per_step": 1e3 * el / steps,
        "gram_ms": 1e3 * t_gram,
        "gram_fp64_equivalent_tflops": gram_flops / t_gram / 1e12,
        "moduli": len(mods),
        "bits_per_column": bits,
        "int8_ops_per_gram": int8_ops,
        "int8_tops_incl_residues_and_reconstruction": int8_ops / t_gram / 1e12,
        "int8_peak_tops": PEAK_INT8_TOPS,
        "max_abs_R_val_final": final,
        "fp64_max_abs_R_val_final": fp64_final,
        "theta_rel_diff_vs_fp64": float(torch.linalg.norm(theta - fp64_theta) / torch.linalg.norm(fp64_theta)),
    }


def lm_comparison(inp, theta0, mu, steps, target):
    """Levenberg-Marquardt damping (gn_step_lm) from the same start as the
    fixed-damping run: steps/s counting every step (a step may factor the
    damped system several times), factorisations and rejected trials, and the
    steps and time to reach the fixed-damping run's final validation
    max-norm (within 5%)."""
    import torch

    from paper_2509_14185_amd import gn

    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    theta = torch.from_numpy(theta0.copy()).cuda()
    prob.step_lm(theta.clone(), mu)  # warm-up on a copy
    torch.cuda.synchronize()
    m_k, tries, done, reached, t_reached = mu, 0, 0, None, None
    elapsed = 0.0
    for k in range(steps):
        t0 = time.perf_counter()
        st = prob.step_lm(theta, m_k)
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        tries += st["tries"]
        done += 1
        m_k = st["mu"]
        if st["rc"] != gn.GN_OK:
            break
        if reached is None and prob.eval(theta)["max_abs_R_val"] <= 1.05 * target:
            reached, t_reached = k + 1, elapsed
    ev = prob.eval(theta)
    prob.close()
    return {
        "value": done / elapsed,
        "unit": "steps/s",
        "ms_per_step": 1e3 * elapsed / done,
        "steps": done,
        "factorisations": tries,
        "rejected_trials": tries - done if st["rc"] == gn.GN_OK else tries - done + 1,
        "mu_initial": mu,
        "mu_final": m_k,
        "last_status": st["rc"],
        "max_abs_R_val_final": ev["max_abs_R_val"],
        "half_sq_norm_final": ev["half_sq_norm"],
        "target_max_abs_R_val": target,
        "steps_to_target": reached,
        "time_to_target_s": t_reached,
    }


def rank1_comparison(inp, theta0, steps, target, period=10, beta=0.95, gamma=1e-3):
    """The paper's stochastic full-matrix GN (gn_step_rank1: moving average of
    rank-1 curvature estimates, factor refreshed every `period` steps,
    closed-form learning rate and momentum) from the same start: steps/s,
    the time of refresh and plain steps, and the steps and time to reach the
    exact-Gram run's final validation max-norm (within 5%).  Probe signs are
    drawn before the timed region."""
    import numpy as np
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    P, m = prob.P, prob.m
    vs = torch.from_numpy(np.stack([workloads.rademacher(m, 1000 + k) for k in range(steps)])).cuda()
    theta = torch.from_numpy(theta0.copy()).cuda()
    G = torch.zeros((P, P), dtype=torch.float64, device="cuda")
    prev = torch.zeros(P, dtype=torch.float64, device="cuda")
    prob.step_rank1(theta.clone(), G.clone(), prev.clone(), vs[0], beta, gamma, True)  # warm-up on copies
    torch.cuda.synchronize()
    t_ref, t_plain, n_ref, reached, t_reached, elapsed = 0.0, 0.0, 0, None, None, 0.0
    for k in range(steps):
        refactor = k % period == 0
        t0 = time.perf_counter()
        st = prob.step_rank1(theta, G, prev, vs[k], beta, gamma, refactor)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        elapsed += dt
        if refactor:
            t_ref, n_ref = t_ref + dt, n_ref + 1
        else:
            t_plain += dt
        if st["rc"] != gn.GN_OK:
            break
        if reached is None and prob.eval(theta)["max_abs_R_val"] <= 1.05 * target:
            reached, t_reached = k + 1, elapsed
    ev = prob.eval(theta)
    prob.close()
    done = k + 1
    return {
        "value": done / elapsed,
        "unit": "steps/s",
        "ms_per_step": 1e3 * elapsed / done,
        "ms_per_refresh_step": 1e3 * t_ref / max(n_ref, 1),
        "ms_per_plain_step": 1e3 * t_plain / max(done - n_ref, 1),
        "steps": done,
        "refresh_period": period,
        "beta": beta,
        "gamma": gamma,
        "last_status": st["rc"],
        "max_abs_R_val_final": ev["max_abs_R_val"],
        "half_sq_norm_final": ev["half_sq_norm"],
        "target_max_abs_R_val": target,
        "steps_to_target": reached,
        "time_to_target_s": t_reached,
    }


def deriv_rows_bench(inp, steps, mu):
    """The medium CCF workload with d1 and d2 rows (N/4 points each): steps/s,
    phases, the Gram rate, and the validation maxima of R, R' and R'' before
    and after, with the blow-up rate implied at the origin."""
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    n1 = n2 = inp["n"] // 4
    s1, s2 = workloads.derivative_points(n1, n2)
    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"], s1=s1, s2=s2)
    P, m = prob.P, prob.m
    theta = torch.from_numpy(inp["theta0"].copy()).cuda()
    ev0, dv0 = prob.eval(theta), prob.eval_derivs(theta)
    prob.step(theta.clone(), mu, stats=False)  # warm-up on a copy
    torch.cuda.synchronize()
    prob.profile_enable(True, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    ev1, dv1 = prob.eval(theta), prob.eval_derivs(theta)
    lam_hat, du0 = prob.lambda_estimate(theta)
    prob.close()
    t_gram = phases["gram"] / nrec * 1e-3
    return {
        "value": steps / el,
        "unit": "steps/s",
        "ms_per_step": 1e3 * el / steps,
        "rows": m,
        "d1_points": n1,
        "d2_points": n2,
        "gram_tflops": float(m) * (P + 1) * (P + 2) / t_gram / 1e12,
        "phase_ms_per_step": {k: v / nrec for k, v in phases.items()},
        "max_abs_R_val": [ev0["max_abs_R_val"], ev1["max_abs_R_val"]],
        "max_abs_dR_val": [dv0[0], dv1[0]],
        "max_abs_d2R_val": [dv0[1], dv1[1]],
        "lambda_hat_final": lam_hat,
        "lambda": inp["lam"],
    }


def funnel_bench(outer=8, steps=50, dlam=0.005, y_max=1.0, pre=300):
    """Funnel inference of lam on the small CCF workload: `pre` GN steps at
    lam_0 = lam - 0.02 from the Glorot start, then up to `outer` trainings of
    `steps` GN steps each, lam moved by the secant on the signed validation
    residual of largest magnitude over y <= y_max (lam kept in (0.3, 1))."""
    import torch

    import workloads
    from paper_2509_14185_amd import funnel, gn

    inp = workloads.make_inputs("ccf_small")
    lam0 = inp["lam"] - 0.02

    def make(lam):
        p = gn.Problem(inp["equation"], inp["widths"], lam, inp["c_norm"], inp["c_target"])
        p.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
        return p

    theta = torch.from_numpy(inp["theta0"].copy()).cuda()
    p0 = make(lam0)
    for _ in range(pre):
        p0.step(theta, inp["mu"], stats=False)
    p0.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lams, rs, ys = funnel.funnel_inference(make, theta, lam0, dlam, outer, steps, inp["mu"], y_max,
                                           lam_range=(0.3, 1.0))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    P = sum(w * (a + 1) for a, w in zip(inp["widths"][:-1], inp["widths"][1:]))
    return {"workload": "ccf_small", "params": P, "pre_steps": pre, "outer": outer, "trainings": len(lams),
            "steps_per_lam": steps, "dlam": dlam, "y_max": y_max, "lam_0": lam0, "lams": lams, "r_hat": rs,
            "y_at": ys, "seconds": el, "ms_per_step": 1e3 * el / max(1, len(lams) * steps)}


def batched_comparison(steps):
    """Batched CCF workload (independent instances with their own lambda and
    point count, shared widths): batched steps (gn_step_batched) against the
    same instances stepped one after another with gn_step."""
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    inps = workloads.make_batched_inputs()
    mu = inps[0]["mu"]
    pgs = []
    for x in inps:
        p = gn.Problem(x["equation"], x["widths"], x["lam"], x["c_norm"], x["c_target"])
        p.set_points(x["s"], x["rho"], x["f"], x["sq"], x["wq"], x["sval"])
        pgs.append(p)
    batch = gn.Batch(pgs)
    ts = [torch.from_numpy(x["theta0"].copy()).cuda() for x in inps]
    init = [p.eval(t)["max_abs_R_val"] for p, t in zip(pgs, ts)]
    batch.step(ts, mu, stats=False)  # warm-up
    torch.cuda.synchronize()
    pgs[0].profile_enable(True, steps)  # the batch records its phases on the first handle
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.step(ts, mu, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases, nrec = pgs[0].profile_read()
    pgs[0].profile_enable(False)
    final = [p.eval(t)["max_abs_R_val"] for p, t in zip(pgs, ts)]
    us = [torch.from_numpy(x["theta0"].copy()).cuda() for x in inps]
    for p, u in zip(pgs, us):
        p.step(u, mu, stats=False)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for p, u in zip(pgs, us):
            p.step(u, mu, stats=False)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    batch.close()
    for p in pgs:
        p.close()
    n = len(inps)
    P1 = inps[0]["P"] + 1
    fl_gram = float(sum((x["n"] + 1) * P1 * (P1 + 1) for x in inps))
    fl_chol = n * P1 ** 3 / 3.0
    t_gram = phases["gram"] / nrec * 1e-3
    t_chol = phases["cholesky"] / nrec * 1e-3
    return {
        "workload": "ccf_batched",
        "roofline": {"bound": "mfma", "kernel": ("batched gram (dgemm_mfma_kernel<128,128,32,1,0,true,512>; the last rows of a bordered "
                                                       "order at most 32 above a multiple of 128 on <32,128,32,1,0,true,512>)"),
                     "achieved": fl_gram / t_gram / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": fl_gram / t_gram / 1e12 / PEAK_FP64_TFLOPS, "traffic": None,
                     "flops_per_step": fl_gram},
        "gram_cholesky_frac": (fl_gram + fl_chol) / (t_gram + t_chol) / 1e12 / PEAK_FP64_TFLOPS,
        "phase_ms_per_step": {k: v / nrec for k, v in phases.items()},
        "instances": n,
        "params": inps[0]["P"],
        "rows_total": int(sum(x["n"] + 1 for x in inps)),
        "steps": steps,
        "batch_steps_per_s": steps / el,
        "instance_steps_per_s": n * steps / el,
        "sequential_instance_steps_per_s": n * steps / el_seq,
        "speedup_vs_sequential": el_seq / el,
        "max_abs_R_val_initial_median": float(sorted(init)[n // 2]),
        "max_abs_R_val_final_median": float(sorted(final)[n // 2]),
    }


def bench_2d(name, steps, warmup, precision="fp64", damping="fixed"):
    """A 2D workload (IPM-style or Boussinesq-type stand-in): steps/s and the
    Gram + Cholesky FP64 fraction.  With row chunks the Jacobian rows are
    formed chunk by chunk between the Gram updates, so the "gram" phase then
    includes the Jacobian sweeps.  damping "lm": Levenberg-Marquardt steps
    from the workload's damping (the phases then cover every factorisation,
    and the objective after each step is recorded)."""
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    inp = workloads.make_inputs_2d(name)
    mu = inp["mu"]
    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"],
                      precision=precision, row_chunk=inp.get("row_chunk", 0))
    prob.set_points_2d(inp["s"], inp["s1"] if inp["n1"] else None, inp["se"], inp["sval"])
    P, m = prob.P, prob.m
    theta = torch.from_numpy(inp["theta0"].copy()).cuda()
    print(f"[bench] {name} ({precision}): P={P} m={m}; warmup {warmup}, {steps} steps", file=sys.stderr, flush=True)
    ev0 = prob.eval(theta)
    lm = damping == "lm"
    for _ in range(warmup):
        if lm:
            prob.step_lm(theta.clone(), mu)
        else:
            prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    prob.profile_enable(True, steps)
    trace, tries, mu_k, failed, mus, tries_k = [], 0, mu, 0, [], []
    t0 = time.perf_counter()
    for k in range(steps):
        # every step reports its status (one synchronisation per step; 2D steps are long)
        if lm:
            st = prob.step_lm(theta, mu_k)
            mu_k, tries = st["mu"], tries + st["tries"]
            trace.append(st["half_sq_norm_new"])
            mus.append(mu_k)
            tries_k.append(st["tries"])
        else:
            st = prob.step(theta, mu)
        failed += int(st["rc"] != gn.GN_OK)
        if steps > 3:
            continue
        torch.cuda.synchronize()
        print(f"[bench] {name} step {k + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    ev1 = prob.eval(theta)
    prob.close()
    fl_gram = float(m) * (P + 1) * (P + 2)
    fl_chol = (P + 1) ** 3 / 3.0
    t_gram = phases["gram"] / nrec * 1e-3
    t_chol = phases["cholesky"] / nrec * 1e-3
    res = {
        "metric": METRIC,
        "value": steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True,
        "dtype": {"fp64": "f64", "split32": "f64 (Gram products f32 hi/lo)",
                  "int8crt": "f64 (Gram from int8 modular products of b-bit column roundings; g and r^T r FP64)"}[precision],
        "data": "synthetic",
        "config": {
            "workload": name,
            "equation": inp["equation"],
            "widths": inp["widths"],
            "params": P,
            "rows": m,
            "collocation_points": inp["n"],
            "d1_points": inp["n1"],
            "boundary_points": inp["ne"],
            "validation_points": int(len(inp["sval"])),
            "row_chunk": inp.get("row_chunk", 0),
            "lam": inp["lam"],
            "mu": mu,
            "precision": precision,
            "max_abs_R_val_initial": ev0["max_abs_R_val"],
            "max_abs_R_val_final": ev1["max_abs_R_val"],
            "half_sq_norm_initial": ev0["half_sq_norm"],
            "half_sq_norm_final": ev1["half_sq_norm"],
            "damping": damping,
            "failed_steps": failed,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": ("gram (dgemm_mfma_kernel<128,128,16,1,0,false,256> on the XCD-balanced work plan, "
                       "accumulated over row chunks; the phase includes the Jacobian sweeps of each chunk)"
                       if inp.get("row_chunk", 0) else
                       "gram (dgemm_mfma_kernel<128,128,16,1,0,false,256> on the XCD-balanced work plan)"),
            "achieved": fl_gram / t_gram / 1e12,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": fl_gram / t_gram / 1e12 / PEAK_FP64_TFLOPS,
            "traffic": None,
            "flops_per_step": fl_gram,
        },
        "gram_tflops": fl_gram / t_gram / 1e12,
        "gram_frac": fl_gram / t_gram / 1e12 / PEAK_FP64_TFLOPS,
        "gram_cholesky_frac": (fl_gram + fl_chol) / (t_gram + t_chol) / 1e12 / PEAK_FP64_TFLOPS,
        "phase_ms_per_step": {k: v / nrec for k, v in phases.items()},
    }
    if lm:
        # the "cholesky" phase then spans every trial: factorisations and trial residuals
        res["lm"] = {"factorisations": tries, "mu_final": mu_k, "half_sq_norm_after_each_step": trace,
                     "factorisations_each_step": tries_k, "mu_after_each_step": mus}
        res["gram_cholesky_frac"] = (fl_gram + fl_chol * tries / steps) / (t_gram + t_chol) / 1e12 / PEAK_FP64_TFLOPS
    return res


def cpu_baseline(inp, mu):
    """Oracle step time on a bounded sample of the same workload, extrapolated,
    on all host cores and on one core.

    Timed pieces: residual rows and the full Jacobian (numpy); the compensated
    Gram on a row sample (linear in rows); the textbook Cholesky and the
    substitutions at a reduced order (cubic / quadratic in order)."""
    import numpy as np

    from oracle import dense
    from oracle import gn as ogn
    from oracle import profile1d as p1

    po = p1.Problem.from_inputs(inp)
    theta = inp["theta0"]
    P, m = po.P, po.m
    all_cores = dense.num_threads()

    def run(rows, order):
        t = {}
        t0 = time.perf_counter()
        r = p1.residual_rows(po, theta)
        t["residual"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        J = p1.jacobian(po, theta)
        t["jacobian"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        dense.gram(J[:rows])
        dense.gradient(J[:rows], r[:rows])
        t["gram"] = (time.perf_counter() - t0) * m / rows
        A = J[:, :order].T @ J[:, :order]
        b = J[:, :order].T @ r
        t0 = time.perf_counter()
        ogn.damped_solve(A, b, mu)
        t["solve"] = (time.perf_counter() - t0) * (P / order) ** 3
        return t

    t_all = run(512, 3072)
    # the small workload's whole 10-step trajectory, measured (no extrapolation)
    import workloads

    sm = workloads.make_inputs("ccf_small")
    ps = p1.Problem.from_inputs(sm)
    th = sm["theta0"]
    t0 = time.perf_counter()
    for _ in range(sm["steps"]):
        th, _ = ogn.step(ps, th, sm["mu"])
    t_small = time.perf_counter() - t0
    dense.set_num_threads(1)
    try:
        t_one = run(32, 1024)
    finally:
        dense.set_num_threads(all_cores)
    sec, sec1 = sum(t_all.values()), sum(t_one.values())
    return {
        "value": 1.0 / sec,
        "unit": "steps/s",
        "cores": all_cores,
        "kind": "oracle",
        "single_core_value": 1.0 / sec1,
        "sample": (f"full residual and Jacobian ({m}x{P}); compensated Gram+gradient on 512 of {m} rows scaled "
                   f"x{m / 512:.0f}; Cholesky+substitutions at order 3072 scaled by (P/3072)^3; seconds per step "
                   f"by part: " + ", ".join(f"{a}={b:.2f}" for a, b in t_all.items()) +
                   f"; one core: Gram on 32 rows, solve at order 1024: " +
                   ", ".join(f"{a}={b:.2f}" for a, b in t_one.items())),
        "ccf_small": {"value": sm["steps"] / t_small, "unit": "steps/s", "cores": all_cores,
                      "sample": f"the whole {sm['steps']}-step trajectory of the small workload, measured"},
    }


def small_bench(mu=None):
    """The small CCF workload's 10-step trajectory (network [1, 32, 32, 1],
    P = 1153, N = 1024 uniform points): steps/s of the 10 steps from the
    Glorot start (one synchronisation at the end), the validation max-norm
    before and after, and the phases."""
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    inp = workloads.make_inputs("ccf_small")
    mu = inp["mu"] if mu is None else mu
    steps = inp["steps"]
    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    P, m = prob.P, prob.m
    theta = torch.from_numpy(inp["theta0"].copy()).cuda()
    for _ in range(3):
        prob.step(theta.clone(), mu, stats=False)  # warm-up on copies
    ev0 = prob.eval(theta)
    torch.cuda.synchronize()
    prob.profile_enable(True, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    ev1 = prob.eval(theta)
    prob.close()
    fl = flops(P, m, inp["n"], inp["m_quad"])
    t_gram = phases["gram"] / nrec * 1e-3
    t_chol = phases["cholesky"] / nrec * 1e-3
    return {
        "workload": "ccf_small",
        "value": steps / el,
        "unit": "steps/s",
        "ms_per_step": 1e3 * el / steps,
        "steps": steps,
        "params": P,
        "rows": m,
        "max_abs_R_val_initial": ev0["max_abs_R_val"],
        "max_abs_R_val_final": ev1["max_abs_R_val"],
        "phase_ms_per_step": {k: v / nrec for k, v in phases.items()},
        "roofline": {"bound": "mfma", "kernel": ("gram (dgemm_mfma_kernel<64,64,32,1,0,false,512> on the XCD-balanced "
                                                    "work plan, then gram_sum_kernel over the tiles split along K)"),
                     "achieved": fl["gram"] / t_gram / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": fl["gram"] / t_gram / 1e12 / PEAK_FP64_TFLOPS, "traffic": None},
        "gram_cholesky_frac": (fl["gram"] + fl["cholesky"]) / (t_gram + t_chol) / 1e12 / PEAK_FP64_TFLOPS,
        "note": "latency-bound: 1.36 GF of Gram and 0.51 GF of Cholesky per step",
    }


def ceilings():
    """Measured ceilings beside the published peaks: FP64 matrix-instruction
    throughput (gn_probe_fp64_mfma: independent MFMA chains, no memory) and a
    1 GiB device-to-device copy (bytes read + written over the copy time)."""
    import torch

    from paper_2509_14185_amd import gn

    mfma = max(gn.probe_fp64_mfma() for _ in range(3))
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 0.0
    for _ in range(5):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * n * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return {"fp64_mfma_spec_tflops": PEAK_FP64_TFLOPS, "fp64_mfma_measured_tflops": mfma,
            "hbm_spec_gbs": PEAK_HBM_GBS, "hbm_copy_measured_gbs": best}


PAPER_FIGURE = {
    "figure": "about 3 GPU-hours for 50k iterations (about 4.6 iterations/s) to a maximum residual of order 1e-8 "
              "on the first unstable CCF profile",
    "hardware": "1x NVIDIA A100",
    "algorithm": "a different optimizer: moving average of rank-1 Gauss-Newton estimates with closed-form learning "
                 "rate and momentum (the rank1 entry here), not the exact damped step timed in value",
    "source": "Methods, Second-order Optimizer, and the main text's CCF results",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pretrain", type=int, default=30,
                    help="untimed FP64 steps before the warm-up, past the transient of the Glorot start")
    ap.add_argument("--workload", default="ccf_medium")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision comparison")
    ap.add_argument("--no-int8", action="store_true", help="skip the int8 modular Gram run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched CCF workload")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D IPM-style workload")
    ap.add_argument("--no-bouss", action="store_true", help="skip the 2D Boussinesq-type workload (about 70 s)")
    ap.add_argument("--no-lm", action="store_true", help="skip the Levenberg-Marquardt runs")
    ap.add_argument("--no-rank1", action="store_true", help="skip the stochastic (rank-1 estimate) run")
    ap.add_argument("--no-deriv", action="store_true", help="skip the run with d1/d2 rows")
    ap.add_argument("--no-funnel", action="store_true", help="skip the funnel-inference run")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the MFMA and copy ceiling probes")
    ap.add_argument("--no-small", action="store_true", help="skip the small-workload trajectory")
    ap.add_argument("--damping", default="fixed", choices=["fixed", "lm"],
                    help="damping of the steps for --workload ipm2d / bouss2d")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split32", "int8crt"],
                    help="arithmetic of the Gram for --workload ipm2d / bouss2d")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; row sharding of the Gram over "
                                   "several GPUs is designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2509_14185_amd import gn

    if args.workload == "ccf_batched":
        # the batched workload alone (its figures also appear under "batched" in the default run)
        print(json.dumps(batched_comparison(args.steps)), flush=True)
        return
    if args.workload in ("ipm2d", "bouss2d"):
        print(json.dumps(bench_2d(args.workload, args.steps, args.warmup, args.precision, args.damping)), flush=True)
        return
    inp = workloads.make_inputs(args.workload)
    mu = inp["mu"]
    prob = gn.Problem(inp["equation"], inp["widths"], inp["lam"], inp["c_norm"], inp["c_target"])
    prob.set_points(inp["s"], inp["rho"], inp["f"], inp["sq"], inp["wq"], inp["sval"])
    P, m, n, mq = prob.P, prob.m, inp["n"], inp["m_quad"]
    theta = torch.from_numpy(inp["theta0"].copy()).cuda()
    print(f"[bench] {args.workload}: P={P} m={m} N={n} M={mq}; pretrain {args.pretrain}, warmup {args.warmup}",
          file=sys.stderr, flush=True)

    ev_glorot = prob.eval(theta)
    for _ in range(args.pretrain + args.warmup):
        prob.step(theta, mu, stats=False)
    theta_start = theta.cpu().numpy()
    ev0 = prob.eval(theta)
    torch.cuda.synchronize()
    prob.profile_enable(True, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prob.step(theta, mu, stats=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases, nrec = prob.profile_read()
    prob.profile_enable(False)
    ev1 = prob.eval(theta)
    last = prob.step(theta.clone(), mu)  # status of one more step from the final iterate
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s; phases (ms total) {phases}", file=sys.stderr, flush=True)

    fl = flops(P, m, n, mq)
    t_gram = phases["gram"] / nrec * 1e-3
    t_chol = phases["cholesky"] / nrec * 1e-3
    gram_tf = fl["gram"] / t_gram / 1e12
    target = ev1["max_abs_R_val"]
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "equation": inp["equation"],
            "widths": inp["widths"],
            "params": P,
            "rows": m,
            "collocation_points": n,
            "hilbert_nodes": mq,
            "points": inp["points"],
            "lam": inp["lam"],
            "mu": mu,
            "precision": "fp64",
            "pretrain_steps": args.pretrain,
            "max_abs_R_val_glorot": ev_glorot["max_abs_R_val"],
            "max_abs_R_val_initial": ev0["max_abs_R_val"],
            "max_abs_R_val_final": ev1["max_abs_R_val"],
            "half_sq_norm_initial": ev0["half_sq_norm"],
            "half_sq_norm_final": ev1["half_sq_norm"],
            "last_step_status": last["rc"],
        },
        "roofline": {
            "bound": "mfma",
            "kernel": ("gram (dgemm_mfma_kernel<128,128,16,1,0,false,256> on the XCD-balanced work plan, "
                       "then gram_sum_kernel over the tiles split along K)"),
            "achieved": gram_tf,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": gram_tf / PEAK_FP64_TFLOPS,
            "traffic": gram_traffic(),
            "traffic_unit": "bytes per launch",
        },
        "gram_cholesky_frac": (fl["gram"] + fl["cholesky"]) / (t_gram + t_chol) / 1e12 / PEAK_FP64_TFLOPS,
        "phase_ms_per_step": {k: v / nrec for k, v in phases.items()},
        "paper_reference": PAPER_FIGURE,
    }
    if not args.no_ceilings:
        print("[bench] measured ceilings", file=sys.stderr, flush=True)
        out["ceilings"] = ceilings()
        out["roofline"]["frac_of_measured_mfma"] = gram_tf / out["ceilings"]["fp64_mfma_measured_tflops"]
    if not args.no_small:
        print("[bench] small CCF trajectory", file=sys.stderr, flush=True)
        out["ccf_small"] = small_bench()
    if not args.no_int8:
        print("[bench] int8 modular Gram", file=sys.stderr, flush=True)
        out["int8crt"] = int8crt_comparison(inp, theta_start, mu, args.steps, theta, target, fl["gram"])
    if not args.no_split:
        print("[bench] split-precision Gram", file=sys.stderr, flush=True)
        out["split32"] = split_comparison(inp, theta_start, mu, args.steps, target, elapsed)
    if not args.no_lm:
        print("[bench] Levenberg-Marquardt damping", file=sys.stderr, flush=True)
        out["lm"] = lm_comparison(inp, theta_start, mu, args.steps, target)
    if not args.no_deriv:
        print("[bench] d1/d2 rows", file=sys.stderr, flush=True)
        out["d12"] = deriv_rows_bench(inp, 10, mu)
    if not args.no_funnel:
        print("[bench] funnel inference", file=sys.stderr, flush=True)
        out["funnel"] = funnel_bench()
    if not args.no_rank1:
        print("[bench] stochastic full-matrix GN (rank-1 estimates)", file=sys.stderr, flush=True)
        out["rank1"] = rank1_comparison(inp, theta_start, 3 * args.steps, target)
        out["rank1"]["paper_reference"] = PAPER_FIGURE["figure"] + " (" + PAPER_FIGURE["hardware"] + ")"
    if not args.no_batched:
        print("[bench] batched CCF workload", file=sys.stderr, flush=True)
        out["batched"] = batched_comparison(10)
    if not args.no_2d:
        r2 = bench_2d("ipm2d", 5, 1)
        out["ipm2d"] = {k: r2[k] for k in ("value", "unit", "ms_per_step", "roofline", "gram_tflops", "gram_frac",
                                            "gram_cholesky_frac", "phase_ms_per_step")}
        out["ipm2d"]["config"] = {k: r2["config"][k] for k in ("widths", "params", "rows", "max_abs_R_val_initial",
                                                               "max_abs_R_val_final", "half_sq_norm_initial",
                                                               "half_sq_norm_final", "mu")}
        if not args.no_int8:
            r8 = bench_2d("ipm2d", 5, 1, precision="int8crt")
            out["ipm2d_int8crt"] = {k: r8[k] for k in ("value", "unit", "ms_per_step", "gram_tflops", "phase_ms_per_step")}
            out["ipm2d_int8crt"]["gram_tflops_note"] = "FP64-equivalent (FP64 Gram flops / int8 Gram time)"
            out["ipm2d_int8crt"]["half_sq_norm_final"] = r8["config"]["half_sq_norm_final"]
            out["ipm2d_int8crt"]["fp64_half_sq_norm_final"] = r2["config"]["half_sq_norm_final"]
        if not args.no_lm:
            r3 = bench_2d("ipm2d", 5, 1, damping="lm")
            out["ipm2d_lm"] = {k: r3[k] for k in ("value", "unit", "ms_per_step", "lm")}
            out["ipm2d_lm"]["config"] = {k: r3["config"][k] for k in ("max_abs_R_val_initial", "max_abs_R_val_final",
                                                                      "half_sq_norm_initial", "half_sq_norm_final",
                                                                      "mu")}
    if not args.no_bouss:
        r5 = bench_2d("bouss2d", 2, 0)
        out["bouss2d"] = {k: r5[k] for k in ("value", "unit", "ms_per_step", "steps", "roofline", "gram_tflops",
                                              "gram_frac", "gram_cholesky_frac", "phase_ms_per_step")}
        out["bouss2d"]["config"] = {k: r5["config"][k] for k in ("widths", "params", "rows", "row_chunk", "mu",
                                                                 "half_sq_norm_initial", "half_sq_norm_final",
                                                                 "max_abs_R_val_initial", "max_abs_R_val_final",
                                                                 "failed_steps")}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inp, mu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
