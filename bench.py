"""Benchmark: simultaneous multi-rhs x multi-shift twisted-mass solves on one MI355X.

Workload: 16^3x32 lattice, seeded links exp(i 0.3 H), kappa = 0.150, 12 Z2-noise
right-hand sides x 4 twisted masses {0.002, 0.01, 0.03, 0.1} = 48 columns.
One step = one ddamg_solve of all 48 columns to a true FP64 relative residual
<= 1e-10 per column (flexible GMRES in FP64, FP32 preconditioner).  The
right-hand sides are resident in HBM before the timed region; the context
(gauge field in the internal layouts, autotuned tile shapes) is built once
before it, as it is shared by every solve on this gauge field.

Printed JSON: value = converged rhs x shift solves per second of the tuned
form; the plain FP64 GPU form of the same method; the roofline of the
dominant kernel measured live with HIP events on the library's stream; the
same workload with a clover term (c_sw = 1.0); and the FP64 oracle timed on
the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "tm_16x16x16x32_12rhs_4shift"

# Solver of the plain FP64 form: FP64 FGMRES(40) preconditioned by FP64 SAP.
# At kappa = 0.150 these seeded fields are past the critical hopping
# parameter; the measured study (see the design notes) found that SAP with one
# red-black cycle and 12 block-MR steps preconditions best, and that the
# aggregation hierarchy does not reduce the outer iteration count there.
SOLVER = dict(n_levels=1, sap_cycles=1, sap_mr_iters=12, outer_restart=40, max_outer=3000)
# The tuned form: FP64 FGMRES(4) whose every step is an FP32 inner FGMRES of
# up to 40 steps (to 1e-2, Arnoldi basis stored in FP16) around FP32 SAP whose
# block solves take 4 MR steps on the odd-even reduced block systems (the
# measured optimum: as few FGMRES steps as 10 MR steps on the full blocks);
# the outer FP64 iteration wins the accuracy back, and its restart every 4
# steps lets converged columns leave the batch.
TUNED = dict(SOLVER, outer_restart=4, inner_iters=40, inner_tol=1e-2, inner_fp16=1, sap_mr_iters=4, sap_oddeven=1)
# the clover form: odd-even block solves are for the clover-free operator, so
# its SAP takes 10 MR steps on the full blocks
CLOVER_SOLVER = dict(TUNED, sap_oddeven=0, sap_mr_iters=10)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "k_sap_oe_fp32_16x16x16x32_48col.md")
# the FP32 SAP half-sweep kernel of each autotuner variant (4^4 blocks) as it
# runs inside the inner Krylov solve, and the time_op form that launches it:
# variants 2 (2-row links) and 3 (full links) read their right-hand side
# straight from the FP16 Arnoldi basis (op 6; the profiler lists those
# instantiations by their mangled names); with odd-even block solves one
# kernel (2-row links) serves every variant
SAP_KERNELS = {0: ("k_sap_half<float, 2, 2, 256, true, float, false>", 1),
               1: ("k_sap_half<float, 2, 2, 256, false, float, false>", 1),
               2: ("_ZN5ddamg10k_sap_halfIfLi2ELi1ELi256ELb0EDF16_Lb0EEE", 6),
               3: ("_ZN5ddamg10k_sap_halfIfLi1ELi1ELi256ELb0EDF16_Lb0EEE", 6)}
SAP_OE_KERNEL = ("_ZN5ddamg8k_sap_oeIfLi2EDF16_Li2EEE", 6)


def sap_kernel(solver, variant):
    """(kernel name, time_op form) of the SAP half sweep a solver runs."""
    if solver.get("sap_oddeven"):
        return SAP_OE_KERNEL
    return SAP_KERNELS[variant]
KERNEL_SOURCE = os.path.join(ROOT, "paper_2201_03872_amd", "csrc", "fine.hip")
# SAP calls timed for the roofline (after one untimed call)
SAP_TIMED_CALLS = 10
# clover coefficient of the twisted-mass clover form measured beside the headline
CLOVER_CSW = 1.0


def measured_traffic(kernel):
    """HBM bytes per launch of the SAP half sweep from the committed counter
    summary, valid only for the same kernel variant while its source is
    unchanged (else None)."""
    import hashlib
    try:
        note = open(TRAFFIC_NOTE).read()
    except OSError:
        return None
    digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    keys = ("kernel_source_sha256", "traffic_bytes_per_launch", "kernel:")
    fields = dict(line.split(":", 1) for line in note.splitlines() if line.startswith(keys))
    if fields.get("kernel_source_sha256", "").strip() != digest or fields.get("kernel", "").strip() != kernel:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def sap_oe_flops_per_half_sweep(V, ncol, mr):
    """Algorithmic flops of one half sweep of SAP with odd-even reduced block
    solves, averaged over the two half sweeps of a one-cycle call, counted per
    pair of an even and an odd site of the active blocks (V / 4 pairs):

    * each MR step applies the Schur complement: the in-block hops of the even
      site (6 on average, 165 flop each), D_ee^-1 (72), the in-block hops of
      the odd site, D_oo (72) and the hop sum (48); then the inner products
      (144) and the two axpys (192) on the odd site: 2508;
    * once: the right-hand side r_o - D_oe D_ee^-1 r_e and the back
      substitution of x_e (6 hops, 48 and 72 each: 2220), and the block
      residual (none in the first half sweep; the 2 block-leaving hops of each
      of the two sites in the second: 660, counted once although the kernel
      evaluates the even one twice)."""
    hop = 1320 / 8
    step = 12 * hop + 72 + 72 + 48 + 144 + 192
    per_pair = mr * step + 2 * (6 * hop + 48 + 72) + 0.5 * (2 * 2 * hop)
    return V / 4 * ncol * per_pair


def sap_flops_per_half_sweep(V, ncol, mr, clover=False):
    """Algorithmic flops of one red-black SAP half sweep (half the sites),
    averaged over the two half sweeps of a one-cycle SAP call.

    Each MR step applies the block operator D_BB, whose hops stay inside the
    4^4 block: 6 of a site's 8 on average (each direction loses the quarter
    of the sites on the block face), 165 flop per hop (1320 / 8), plus the
    diagonal (4 flop per real, 96), the two inner products <q, rho> and
    |q|^2 (12 flop per complex, 144) and the two complex axpys (8 flop per
    complex each, 192).  The block residual costs nothing in the first half
    sweep (x = 0, residual = right-hand side); in the second, x is still zero
    inside its own blocks, so only the 2 block-leaving hops per site count.
    With a clover term the site term is two Hermitian 6x6 blocks (6 real
    diagonal entries, 15 complex pairs: 504 flop) plus the twist and the
    hop sum (72) in place of the 96 of the scalar diagonal; the second half
    sweep's residual applies it to x = 0 and is not counted."""
    hop = 1320 / 8
    site = 504 + 72 if clover else 96
    per_site = 0.5 * (2 * hop) + mr * (6 * hop + site + 144 + 192)
    return V / 2 * ncol * per_site


def cpu_baseline(w, U, outer_iters, sap_mr, oddeven=False):
    """The FP64 oracle on a bounded sample of the same workload: one column of
    the 16^3x32 problem, one oracle application of each operation of an outer
    iteration (fine operator, one-cycle SAP, 20-vector Gram-Schmidt step),
    scaled by the FGMRES iteration count (outer + inner) of the GPU solve.  The SAP
    cost is affine in the MR step count; it is timed at 1 and 2 steps and
    extrapolated to the solver's count.  numpy runs on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    import synthetic as S
    from oracle.multigrid import Blocking, FineLevel
    with threadpool_limits(limits=1):
        return _cpu_baseline(w, U, outer_iters, sap_mr, oddeven, np, O, S, Blocking, FineLevel)


def _cpu_baseline(w, U, outer_iters, sap_mr, oddeven, np, O, S, Blocking, FineLevel):
    t_all = time.time()
    lev = FineLevel(O.WilsonTM(U, w.dims, kappa=w.kappa))
    V = w.volume
    x = S.gaussian_spinors(1, V, 1).reshape(1, V, 12)
    mus = np.array([w.mus[0]])

    def timed(f, n=1):
        t = time.time()
        for _ in range(n):
            f()
        return (time.time() - t) / n

    t_fine = timed(lambda: lev.apply(x, mus))
    sb = Blocking(w.dims, w.sap_block)
    t_s1 = timed(lambda: O.sap(lev, sb, x, mus, 1, 1, oddeven=oddeven))
    t_s2 = timed(lambda: O.sap(lev, sb, x, mus, 1, 2, oddeven=oddeven))
    t_sap = t_s1 + (sap_mr - 1) * max(t_s2 - t_s1, 0.0)
    basis = [x * (k + 1) for k in range(20)]

    def gram():
        h = [O.col_dot(b, x) for b in basis]
        y = x.copy()
        for hb, b in zip(h, basis):
            y = y - hb[:, None, None] * b
        return O.col_norm(y)

    t_gram = timed(gram)
    per_col = outer_iters * (t_fine + t_sap + t_gram)
    return dict(value=1.0 / per_col, unit="rhs*shift solves/s", cores=1, kind="oracle",
                sample=(f"one column of {w.name}: one numpy-FP64 oracle application each of the fine operator "
                        f"({t_fine:.2f}s), one-cycle SAP with {sap_mr} MR steps{' (odd-even)' if oddeven else ''} "
                        f"({t_sap:.2f}s, from 1- and 2-step "
                        f"timings {t_s1:.2f}s/{t_s2:.2f}s) and a 20-vector "
                        f"Gram-Schmidt step ({t_gram:.2f}s), times the {outer_iters} FGMRES iterations (outer + "
                        f"inner) the GPU solve needed; sampling took {time.time() - t_all:.0f}s"))


# Learned-smoother study: 16^3x32 fields drawn like the benchmark's (eps 0.3,
# kappa 0.150), 8 training and 4 held-out gauge seeds; 8 x 160 Adam steps of
# 16 residual -> error pairs (20480 pairs), errors from 0..2 SAP sweeps; the
# trained net (4 minimal-residual steps per call, SAP fallback) replaces SAP in
# FGMRES(40) on 3 rhs x 4 shifts per held-out field.
LEARNED_TRAIN_SEEDS = tuple(range(4101, 4109))
LEARNED_HELDOUT_SEEDS = tuple(range(4201, 4205))
LEARNED = dict(steps=160, batch=16, lr=2e-3, sap_sweeps=2, cycles=4, n_rhs=3)


def learned_study(dd, S, np, torch):
    w = S.workload(WORKLOAD)
    mus = np.array(w.mus)
    b = torch.from_numpy(S.rhs_for(w)[:LEARNED["n_rhs"]].copy()).cuda()
    ncol = b.shape[0] * len(mus)
    m0 = 1 / (2 * w.kappa) - 4
    W1 = np.zeros((9, 2, 1, 4, 4), dtype=np.complex128)
    W2 = np.zeros((9, 1, 2, 4, 4), dtype=np.complex128)
    W1[0, 0, 0], W1[0, 1, 0] = np.eye(4), 0.01 * np.eye(4)          # start: f(r) = r / (4 + m0)
    W2[0, 0, 0], W2[0, 0, 1] = np.eye(4) / (4 + m0), 0.01 * np.eye(4)
    weights = (W1, W2)

    def ctx_for(seed, **kw):
        U = S.gauge_field(w.dims, w.eps, seed)
        c = dd.Context(dd.params_for_workload(w, precision=dd.MIXED, **{**SOLVER, **kw}), U)
        c.autotune(ncol)
        return c

    t0 = time.time()
    losses = []
    for k, seed in enumerate(LEARNED_TRAIN_SEEDS):
        c = ctx_for(seed)
        c.set_smoother_weights(*weights)
        h = c.train_smoother(mus, LEARNED["steps"], LEARNED["batch"], LEARNED["lr"], LEARNED["sap_sweeps"],
                             seed=7 + k)
        weights = c.smoother_weights()
        c.close()
        losses.append((float(h[:10].mean()), float(h[-10:].mean())))
        log(f"  trained on gauge seed {seed}: loss {losses[-1][0]:.4f} -> {losses[-1][1]:.4f}")
    torch.cuda.synchronize()
    train_s = time.time() - t0

    def timed_solve(c):
        torch.cuda.synchronize()
        t = time.time()
        x, info, st = c.solve(mus, b)
        torch.cuda.synchronize()
        t = time.time() - t
        ok = st == dd.OK and all(i["converged"] for i in info)
        return dict(iters=max(i["outer_iters"] for i in info), seconds=t, converged=ok,
                    worst_true_rel_res=max(i["true_rel_res"] for i in info))

    rows = []
    for seed in LEARNED_HELDOUT_SEEDS:
        c = ctx_for(seed)
        sap = timed_solve(c)
        c.close()
        c = ctx_for(seed, smoother=dd.SMOOTHER_LEARNED, smoother_cycles=LEARNED["cycles"])
        c.set_smoother_weights(W1, W2)
        untrained = timed_solve(c)
        c.set_smoother_weights(*weights)
        learned = timed_solve(c)
        learned["fallbacks"] = c.stats()["learned_fallbacks"]
        c.close()
        rows.append(dict(seed=seed, sap=sap, learned_untrained=untrained, learned=learned))
        log(f"  held-out seed {seed}: SAP {sap['iters']} it {sap['seconds']:.2f}s, untrained net "
            f"{untrained['iters']} it, trained net {learned['iters']} it {learned['seconds']:.2f}s "
            f"({learned['fallbacks']} fallbacks)")
    mean = lambda key, f: float(np.mean([r[key][f] for r in rows]))
    out = {
        "metric": "outer FGMRES iterations and seconds per solve, learned smoother vs SAP (held-out fields)",
        "value": mean("sap", "seconds") / mean("learned", "seconds"),
        "unit": "SAP time / learned-smoother time",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "dtype": "f64 outer / f32 smoother / bf16 network weights",
        "config": {"workload": "16x16x16x32 learned-smoother study", "kappa": w.kappa, "eps": w.eps,
                   "train_seeds": list(LEARNED_TRAIN_SEEDS), "heldout_seeds": list(LEARNED_HELDOUT_SEEDS),
                   "pairs": len(LEARNED_TRAIN_SEEDS) * LEARNED["steps"] * LEARNED["batch"],
                   "columns": ncol, **LEARNED},
        "train_seconds": train_s, "train_loss": losses,
        "mean_iters": {k: mean(k, "iters") for k in ("sap", "learned_untrained", "learned")},
        "mean_seconds": {k: mean(k, "seconds") for k in ("sap", "learned_untrained", "learned")},
        "all_converged": all(r[k]["converged"] for r in rows for k in ("sap", "learned")),
        "heldout": rows,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-clover", action="store_true", help="skip the twisted-mass clover measurement")
    ap.add_argument("--learned", action="store_true",
                    help="instead of the solve benchmark, train the learned smoother on 8 gauge fields and "
                         "compare it with SAP on 4 held-out fields")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (how it would shard is "
              "described in the design notes); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2201_03872_amd as dd
    import synthetic as S

    torch.cuda.set_device(0)
    dd.load()
    if args.learned:
        learned_study(dd, S, np, torch)
        return
    w = S.workload(WORKLOAD)
    log("workload", w.name, "- generating inputs")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    mus = np.array(w.mus)
    ncol = w.n_col

    def run_form(precision, steps, warmup, solver, time_sap=False):
        p = dd.params_for_workload(w, precision=precision, **solver)
        t0 = time.time()
        ctx = dd.Context(p, U)
        tuned = ctx.autotune(ncol)
        torch.cuda.synchronize()
        setup_s = time.time() - t0
        log(f"  precision={precision}: context + autotune {setup_s:.2f}s {tuned}")
        for i in range(warmup):
            ctx.solve(mus, b)
            log(f"  warmup solve {i} done")
        if time_sap:   # HIP events around every SAP kernel launch of the timed solves
            ctx.set_tuning("time_sap", 1)
        torch.cuda.synchronize()
        t0 = time.time()
        allconv, worst = True, 0.0
        for i in range(steps):
            x, info, st = ctx.solve(mus, b)
            allconv &= all(c["converged"] for c in info)
            worst = max(worst, max(c["true_rel_res"] for c in info))
            log(f"  step {i} done ({time.time() - t0:.2f}s)")
        torch.cuda.synchronize()
        el = time.time() - t0
        stats = ctx.stats()
        if time_sap:
            ctx.set_tuning("time_sap", 0)
        return ctx, dict(setup_s=setup_s, elapsed=el, allconv=allconv, worst=worst, stats=stats, tuned=tuned)

    ctx, tuned = run_form(dd.MIXED, args.steps, args.warmup, TUNED, time_sap=True)
    value = ncol * args.steps / tuned["elapsed"]
    log("tuned form", tuned)

    # roofline of the dominant kernel of the tuned solve (the FP32 SAP half
    # sweep) and of the fine stencil, timed with HIP events on the context stream
    n_iter = 10
    V = w.volume
    sap_name, sap_op = sap_kernel(TUNED, tuned["tuned"]["sap_variant"])
    t_sap = ctx.time_op(sap_op, 0, dd.FP32, ncol, SAP_TIMED_CALLS) / 2.0   # one call = two half sweeps
    sap_flops = (sap_oe_flops_per_half_sweep(V, ncol, TUNED["sap_mr_iters"]) if TUNED.get("sap_oddeven")
                 else sap_flops_per_half_sweep(V, ncol, TUNED["sap_mr_iters"]))
    sap_tf_standalone = sap_flops / t_sap / 1e12
    # the same kernel inside the last timed solve: HIP events around each of its
    # launches on the context stream; the flops scale with the column tiles of
    # each launch (converged tiles leave the batch)
    st_t = tuned["stats"]
    ntile = (ncol + 7) // 8
    sap_ms, sap_n, sap_tiles = st_t["sap_kernel_ms"], st_t["n_sap_kernels"], st_t["n_sap_kernel_tiles"]
    sap_us_solve = sap_ms * 1e3 / sap_n if sap_n else None
    sap_tf_solve = (sap_flops / ntile * sap_tiles) / (sap_ms * 1e-3) / 1e12 if sap_n else None
    t_copy = ctx.time_op(5, 0, dd.FP64, ncol, 5)              # plain copy of one FP64 48-column vector
    copy_bytes = 2 * V * 12 * 16 * ncol
    t32 = ctx.time_op(0, 0, dd.FP32, ncol, n_iter)
    t64 = ctx.time_op(0, 0, dd.FP64, ncol, n_iter)
    links32 = 288 if tuned["tuned"]["fp32_links"] == 0 else 192
    bytes32 = V * (links32 + ncol * 48 * 4)
    bytes64 = V * (576 + ncol * 48 * 8)
    ctx.close()

    # the coarse stencil on the hierarchy of this workload (4^4 then 2^4
    # aggregates, 24 / 32 test vectors): BF16 MFMA against the FP32 vector
    # kernel and FP64, HIP events on the context stream
    cctx = dd.Context(dd.params_for_workload(w, precision=dd.MIXED, setup_rounds=1), U)
    coarse = {}
    for level in (1, 2):
        Vc, dof, cdims = cctx.level_info(level)
        flops = Vc * 9 * dof * dof * 8 * ncol
        row = {"sites": Vc, "dof": dof, "flop_per_launch": flops}
        for name, prec, knob in (("bf16_mfma", dd.FP32, 1), ("fp32_vector", dd.FP32, 0), ("fp64", dd.FP64, 0)):
            cctx.set_tuning("coarse_mfma", knob)
            sec = cctx.time_op(2, level, prec, ncol, 50)
            row[name] = {"us": sec * 1e6, "TFLOPs": flops / sec / 1e12}
        row["bf16_mfma"]["frac_of_bf16_peak"] = row["bf16_mfma"]["TFLOPs"] / 2500.0
        coarse[f"level{level}"] = row
    cctx.close()
    log("coarse stencil", coarse)

    # the twisted-mass clover operator on the same workload and solver
    # (c_sw = CLOVER_CSW): one warm-up and one timed solve, the clover forms
    # of the fine stencil and of the FP16-input SAP half sweep (HIP events)
    clover = None
    if not args.no_clover:
        cctx, cl = run_form(dd.MIXED, 1, 1, dict(CLOVER_SOLVER, csw=CLOVER_CSW))
        log("clover form", cl)
        t32c = cctx.time_op(0, 0, dd.FP32, ncol, n_iter)
        t64c = cctx.time_op(0, 0, dd.FP64, ncol, n_iter)
        _, csap_op = sap_kernel(CLOVER_SOLVER, cl["tuned"]["sap_variant"])
        tsc = cctx.time_op(csap_op, 0, dd.FP32, ncol, SAP_TIMED_CALLS) / 2.0
        cctx.close()
        links32c = 288 if cl["tuned"]["fp32_links"] == 0 else 192
        bytes32c = V * (links32c + 288 + ncol * 48 * 4)      # + the FP32 clover blocks
        bytes64c = V * (576 + 576 + ncol * 48 * 8)
        csap_flops = sap_flops_per_half_sweep(V, ncol, CLOVER_SOLVER["sap_mr_iters"], clover=True)
        clover = {"csw": CLOVER_CSW, "solves_per_s": ncol / cl["elapsed"] if cl["allconv"] else 0.0,
                  "all_converged": cl["allconv"], "worst_true_rel_res": cl["worst"],
                  "outer_iters": cl["stats"]["outer_iters"], "inner_iters": cl["stats"]["n_inner_iters"],
                  "dslash_fp32_us": t32c * 1e6, "dslash_fp32_GBs": bytes32c / t32c / 1e9,
                  "dslash_fp64_us": t64c * 1e6, "dslash_fp64_GBs": bytes64c / t64c / 1e9,
                  "sap_half_sweep_us": tsc * 1e6, "sap_TFLOPs": csap_flops / tsc / 1e12}

    plain = None
    if not args.no_plain:
        pctx, plain = run_form(dd.PLAIN_FP64, 1, 0, SOLVER)
        pctx.close()
        log("plain FP64 form", plain)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle sample")
        cpu = cpu_baseline(w, U, tuned["stats"]["outer_iters"] + tuned["stats"]["n_inner_iters"],
                           TUNED["sap_mr_iters"], bool(TUNED.get("sap_oddeven")))

    sap_tf = sap_tf_solve if sap_tf_solve is not None else sap_tf_standalone
    out = {
        "metric": "rhs*shift solves/s at true FP64 relative residual 1e-10 (tuned form); dslash HBM GB/s",
        "value": value if tuned["allconv"] else 0.0,
        "unit": "rhs*shift solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tuned["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 inner (f16 basis storage) / f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": "16x16x16x32", "kappa": w.kappa, "n_rhs": w.n_rhs,
                   "shifts": list(w.mus), "columns": ncol, "tol": 1e-10,
                   "solver": "FP64 FGMRES(4) over FP32 FGMRES(40, to 1e-2, FP16 basis) over FP32 red-black "
                             "SAP (4^4 blocks, 1 cycle, 4 MR steps on the odd-even reduced blocks)",
                   "plain_solver": "FP64 FGMRES(40) over FP64 red-black SAP (4^4 blocks, 1 cycle, 12 MR steps)"},
        "all_converged": tuned["allconv"],
        "worst_true_rel_res": tuned["worst"],
        "outer_iters": tuned["stats"]["outer_iters"],
        "inner_iters": tuned["stats"]["n_inner_iters"],
        "plain_outer_iters": plain["stats"]["outer_iters"] if plain else None,
        "context_setup_s": tuned["setup_s"],
        "autotuned": tuned["tuned"],
        "plain_fp64_solves_per_s": (ncol / plain["elapsed"]) if plain and plain["allconv"] else None,
        "tuned_over_plain": (value / (ncol / plain["elapsed"])) if plain and plain["allconv"] else None,
        "dslash": {"fp32_us": t32 * 1e6, "fp32_GBs": bytes32 / t32 / 1e9,
                   "fp32_GFLOPs": 1320 * V * ncol / t32 / 1e9,
                   "fp64_us": t64 * 1e6, "fp64_GBs": bytes64 / t64 / 1e9,
                   "fp64_GFLOPs": 1320 * V * ncol / t64 / 1e9,
                   "fp64_hbm_frac": bytes64 / t64 / 1e9 / HBM_PEAK_GBS},
        "roofline": {"kernel": sap_name + " (FP32 red-black SAP half sweep, 48 columns)",
                     "bound": "alu", "achieved": sap_tf, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": sap_tf / 157.3, "traffic": measured_traffic(sap_name),
                     "us_per_launch": sap_us_solve if sap_us_solve is not None else t_sap * 1e6,
                     "launches_timed": sap_n, "timed_in": "the last timed solve" if sap_n else "standalone calls",
                     "standalone": {"us_per_launch": t_sap * 1e6, "achieved": sap_tf_standalone,
                                    "launches": 2 * SAP_TIMED_CALLS}},
        "copy_kernel_GBs": copy_bytes / t_copy / 1e9,
        "coarse_stencil_48col": coarse,
        "clover": clover,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
