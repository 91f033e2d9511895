"""Benchmark: simultaneous multi-rhs x multi-shift twisted-mass solves on one MI355X.

Headline workload: the 40^3x80 lattice (one GPU's share of an 80^3x160 run),
seeded links exp(i 0.35 H), kappa = 0.152, 4 Gaussian right-hand sides x 8
twisted masses log-spaced in [7e-4, 0.5] = 32 columns.  One step = one
ddamg_solve of all 32 columns to a true FP64 relative residual <= 1e-10 per
column.  The right-hand sides are resident in HBM before the timed region;
the context (gauge field in the internal layouts, the multigrid hierarchy,
autotuned tile shapes) is built once before it and shared by every solve on
this gauge field.

Solver (paper sections 2 and 4): FP64 flexible GMRES preconditioned by the
aggregation multigrid cycle with red-black SAP; the coarse solves run GMRES on
the gamma5-Hermitian form of the coarse operator.  The tuned form runs the
cycle in FP32 with the coarse stencil on BF16 MFMA; the plain form runs the
same method in FP64.  Columns are solved 8 at a time (memory), converged
columns leave the batch.

Printed JSON: value = converged rhs x shift solves per second of the tuned
form; the plain FP64 form of the same method; the three-level hierarchy; the
16^3x32 workload in its one-, two- and three-level forms; the roofline of the
dominant kernel measured live with HIP events on the library's stream; the
fine stencil's bandwidth; and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
WORKLOAD = "tm_40x40x40x80_4rhs_8shift"
SMALL = "tm_16x16x16x32_12rhs_4shift"

# Two-level aggregation multigrid (4^4 aggregates, 24 test vectors, one
# bootstrap round), one red-black SAP cycle with 4 MR steps on the odd-even
# reduced 4^4 blocks, coarse GMRES on the gamma5-Hermitian form to 0.1.
MG2 = dict(n_levels=2, sap_cycles=1, sap_mr_iters=4, sap_oddeven=1, setup_rounds=3, setup_boot=1,
           coarse_gamma5=1, bottom_maxit=100, inner_iters=0)
# 40^3x80, 8 columns in flight (HBM budget).  Plain form: FP64 FGMRES(4)
# over the cycle, all in FP64.  Tuned form: FP64 FGMRES(1) over an FP32
# FGMRES(12) to 1e-2 whose basis is stored in FP16, over the FP32 cycle with
# BF16 coarse blocks (the nested solve fits in HBM because its basis is FP16);
# the coarse GMRES basis is stored in FP16 as well and the level-0 transfers
# read P in FP16.
# The 40^3x80 hierarchy and cycle: two setup smoothing rounds and two
# bootstrap rounds, SAP with 5 MR steps, coarse GMRES to 0.15 (the fastest
# settings of parameter sweeps over one 8-column wave and over all 32 columns
# of this workload).
MG2_40 = dict(MG2, setup_rounds=2, setup_boot=2, sap_mr_iters=5, r_b=0.15)
PLAIN = dict(MG2_40, outer_restart=4, max_outer=300, max_active_cols=8)
TUNED = dict(PLAIN, outer_restart=1, inner_iters=12, inner_tol=1e-2, inner_fp16=1, coarse_fp16=1, transfer_fp16=1)
# the three-level hierarchy of the workload definition (4^4 then 2^4
# aggregates, 24 / 32 test vectors): middle FGMRES to 7e-2, coarsest GMRES to 0.1
THREE = dict(PLAIN, n_levels=3, middle_restart=25, middle_maxit=50)
# its coarsest level with a short restart, plain and with deflated restarting
# (GMRES-DR(10, 4): 4 harmonic Ritz vectors kept across restarts)
THREE_R10 = dict(THREE, bottom_restart=10)
THREE_DR = dict(THREE_R10, bottom_dr_k=4)
# 16^3x32 forms: one-level (FP64 FGMRES(4) over an FP32 FGMRES(40) with an FP16
# basis around SAP), two- and three-level (FP64 FGMRES(40) over the cycle)
SMALL_ONE = dict(n_levels=1, sap_cycles=1, sap_mr_iters=4, sap_oddeven=1, outer_restart=4, inner_iters=40,
                 inner_tol=1e-2, inner_fp16=1, max_outer=3000)
SMALL_TWO = dict(MG2, outer_restart=40, max_outer=400)
SMALL_THREE = dict(SMALL_TWO, n_levels=3, middle_restart=25, middle_maxit=50)

# the kernel classes the library can time live (ddamg.h, DDAMG_KNOB_TIME_SAP)
TIMED = {"sap": 1, "coarse1": 2, "restrict0": 3, "prolong0": 4, "dslash": 5}
# roofline kernel of the tuned solve: the FP32 odd-even SAP half sweep, the
# largest share of the solve's kernel time in the committed trace; the level-1
# coarse stencil (BF16 MFMA) is reported beside it
ROOFLINE_CLASS = "sap"


# counter summaries (rocprofv3 FETCH_SIZE / WRITE_SIZE passes calibrated by
# the copy kernel) of the level-1 coarse stencil and of the SAP half sweep
# (the roofline kernel); a traffic figure holds while the kernel's source file
# is the one the counters were taken with
_HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE = os.path.join(_HERE, "profiles", "k_coarse_mfma_t1_48_40x40x40x80_8col.md")
KERNEL_SRC = os.path.join(_HERE, "paper_2201_03872_amd", "csrc", "coarse.hip")
SAP_PROFILE = os.path.join(_HERE, "profiles", "k_sap_oe_fp32_40x40x40x80_8col.md")
SAP_SRC = os.path.join(_HERE, "paper_2201_03872_amd", "csrc", "fine.hip")


def counter_traffic(profile=None, src=None):
    """Calibrated HBM traffic per launch (bytes) of a kernel from its counter
    summary, or None when the summary is missing or the kernel's source file
    has changed since the counters were taken (its SHA-256 is recorded)."""
    import hashlib
    import re
    profile = PROFILE if profile is None else profile
    src = KERNEL_SRC if src is None else src
    try:
        txt = open(profile).read()
        sha = re.search(r"SHA-256 of \S+ when the counters were taken \| ([0-9a-f]{64})", txt).group(1)
        gb = float(re.search(r"traffic per launch \(calibrated fetch \+ write\) \| ([0-9.]+) GB", txt).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
        return None
    return gb * 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def coarse1_bytes_flops(Vc, d, ncol_tiles):
    """Algorithmic bytes and flops of one launch of the level-1 coarse stencil
    on BF16 MFMA: the 9 blocks of each coarse site once in the MFMA operand
    form [Re A | Im A] (d x 2d BF16, 4 d^2 bytes per block), the input vector
    as the coarse GMRES stores it (an FP16 basis vector, 4 bytes per complex;
    the few restart residuals read FP32) and the FP32 output (8 bytes per
    complex), 8 columns per tile; flops 8 per complex multiply-add, 9 d^2 per
    site and column."""
    ncol = 8 * ncol_tiles
    bytes_ = Vc * (9 * 4 * d * d + (4 + 8) * d * ncol)
    flops = Vc * 9 * d * d * 8 * ncol
    return bytes_, flops


def sap_oe_flops_per_tile(V, k_mr):
    """Algorithmic flops of one launch of the odd-even SAP half sweep over one
    8-column tile: per pair of an even and an odd site of the active colour
    (V / 4 pairs) and column, k_mr Schur steps of 12 in-block hops (165 flop
    each: projection, SU(3) products, reconstruction), D_ee^-1 and D_oo (72
    each), the hop sum (48), the inner products (144) and the axpys (192); the
    right-hand side and the back substitution (2 * (6 * 165 + 48 + 72)); the
    block-leaving hops of the block residual (2 per site, second half sweep
    only: counted at half)."""
    per_pair = k_mr * (12 * 165 + 72 + 72 + 48 + 144 + 192) + 2 * (6 * 165 + 48 + 72) + 2 * 2 * 165 // 2
    return (V // 4) * 8 * per_pair


def run_form(dd, torch, w, U, b, mus, precision, solver, steps, warmup_rhs, tune_cols, timed_class=None,
             label=""):
    """Context + autotune, one untimed solve of `warmup_rhs` right-hand sides
    (allocates the workspaces a wave of columns needs), then `steps` timed
    solves of all columns."""
    p = dd.params_for_workload(w, precision=precision, **solver)
    t0 = time.time()
    ctx = dd.Context(p, U)
    t_h = time.time() - t0
    tuned = ctx.autotune(tune_cols)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log(f"  {label}: hierarchy {t_h:.1f}s, context + autotune {setup_s:.1f}s")
    if warmup_rhs:
        ctx.solve(mus, b[:warmup_rhs].contiguous())
        log(f"  {label}: warm-up solve done")
    if timed_class:
        ctx.set_tuning("time_kernel", TIMED[timed_class])
    torch.cuda.synchronize()
    t0 = time.time()
    allconv, worst, iters = True, 0.0, []
    for i in range(steps):
        x, info, st = ctx.solve(mus, b)
        allconv &= all(c["converged"] for c in info)
        worst = max(worst, max(c["true_rel_res"] for c in info))
        iters = [c["outer_iters"] for c in info]
        log(f"  {label}: step {i} done ({time.time() - t0:.2f}s)")
    torch.cuda.synchronize()
    el = time.time() - t0
    stats = ctx.stats()
    if timed_class:
        ctx.set_tuning("time_kernel", 0)
    ncol = len(iters)
    return ctx, dict(setup_s=setup_s, hierarchy_s=t_h, elapsed=el, allconv=allconv, worst=worst, stats=stats,
                     tuned=tuned, outer_iters_max=max(iters), outer_iters_mean=sum(iters) / ncol,
                     solves_per_s=(ncol * steps / el) if allconv else 0.0, x=x)


def summary(r, precision_note):
    s = r["stats"]
    return {"solves_per_s": r["solves_per_s"], "seconds_per_solve_call": r["elapsed"], "all_converged": r["allconv"],
            "worst_true_rel_res": r["worst"], "outer_iters_max": r["outer_iters_max"],
            "outer_iters_mean": r["outer_iters_mean"], "avg_bottom_iters": s["avg_bottom_iters"],
            "n_bottom_solves": s["n_bottom_solves"], "avg_middle_iters": s["avg_middle_iters"],
            "n_middle_solves": s["n_middle_solves"], "inner_iters": s["n_inner_iters"],
            "setup_s": r["setup_s"], "hierarchy_s": r["hierarchy_s"], "precision": precision_note,
            "device_GB_peak": s["device_bytes_peak"] / 1e9}


# --------------------------------------------------------------- CPU baseline ---
def _cpu_c1_column(args):
    """One column of the 4^4 workload solved by the FP64 oracle's two-level
    multigrid (one process, one thread)."""
    c, = args
    from threadpoolctl import threadpool_limits
    import numpy as np
    import oracle as O
    import synthetic as S
    with threadpool_limits(limits=1):
        w = S.workload("tm_4x4x4x4_2rhs_3shift")
        U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
        p = O.MGParams(agg=w.agg, n_tv=w.n_tv, sap_block=w.sap_block, mu_setup=min(w.mus))
        t = time.time()
        mg = O.OracleMG(U, w.dims, w.kappa, p).setup(S.setup_start_vectors(w))
        b = S.rhs_for(w)[c // len(w.mus)][None]
        mu = np.array([w.mus[c % len(w.mus)]])
        x, info = mg.solve(b, mu)
        ok = bool(mg.true_relres(b, x, mu)[0] <= 1e-10)
        return time.time() - t, ok


def _cpu_c5_sample(args):
    """Per-operation FP64 oracle timings of the two-level method on a 8^3x16
    sub-lattice drawn with the 40^3x80 recipe (one process, one thread):
    fine operator, one-cycle odd-even SAP, restriction, prolongation, one
    coarse operator application and a 5-vector Gram-Schmidt step on each
    level.  Every cost is per site and scales with the volume."""
    seed, = args
    from threadpoolctl import threadpool_limits
    import numpy as np
    import oracle as O
    import synthetic as S
    from oracle.multigrid import Blocking, FineLevel, build_prolongator, restrict, prolong, galerkin
    with threadpool_limits(limits=1):
        w = S.workload(WORKLOAD)
        dims = (8, 8, 8, 16)
        U = S.gauge_field(dims, w.eps, w.seed_gauge + seed)
        lev = FineLevel(O.WilsonTM(U, dims, kappa=w.kappa))
        V = lev.V
        x = S.gaussian_spinors(1, V, 1 + seed).reshape(1, V, 12)
        mus = np.array([w.mus[0]])
        sb = Blocking(dims, (4, 4, 4, 4))
        tv = S.gaussian_spinors(24, V, 2 + seed).reshape(24, V, 12)
        P = build_prolongator(tv, sb)
        coarse = galerkin(lev, P, sb)
        xc = restrict(P, sb, x)

        def timed(f, n=3):
            t = time.time()
            for _ in range(n):
                f()
            return (time.time() - t) / n

        def gram(v, k):
            basis = [v * (j + 1) for j in range(k)]
            h = [O.col_dot(bb, v) for bb in basis]
            y = v.copy()
            for hb, bb in zip(h, basis):
                y = y - hb[:, None, None] * bb
            return O.col_norm(y)

        return dict(V=V, Vc=coarse.V,
                    fine_op=timed(lambda: lev.apply(x, mus)),
                    sap=timed(lambda: O.sap(lev, sb, x, mus, 1, 4, oddeven=True), 1),
                    restrict=timed(lambda: restrict(P, sb, x)),
                    prolong=timed(lambda: prolong(P, sb, xc)),
                    coarse_op=timed(lambda: coarse.apply(xc, mus), 10),
                    gram_fine=timed(lambda: gram(x, 5)),
                    gram_coarse=timed(lambda: gram(xc, 17), 10))


def cpu_measure():
    """The FP64 oracle on the host cores, one column per process (all cores
    busy at once), run before the process touches the GPU: (1) the 4^4
    workload's 6 columns solved in full by the oracle's two-level multigrid;
    (2) per-operation oracle timings of the two-level method on 8^3x16
    sub-lattices drawn with the 40^3x80 recipe."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    cpu_model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ctx = mp.get_context("fork")
    t0 = time.time()
    with ctx.Pool(min(cores, 6)) as pool:
        c1 = pool.map(_cpu_c1_column, [(c,) for c in range(6)])
    c1_wall = time.time() - t0
    t0 = time.time()
    with ctx.Pool(cores) as pool:
        samples = pool.map(_cpu_c5_sample, [(k,) for k in range(cores)])
    return dict(cores=cores, cpu_model=cpu_model, c1=c1, c1_wall=c1_wall, samples=samples,
                c5_wall=time.time() - t0)


def cpu_baseline(raw, tuned_stats, outer_per_col, ncol, V_fine, Vc):
    """Combines the oracle timings with the operation counts of the GPU's
    tuned solve: the headline workload's per-column oracle time is the
    per-site operation costs scaled to 40^3x80 times the counts."""
    import numpy as np
    samples, cores = raw["samples"], raw["cores"]
    m = {k: float(np.mean([s[k] for s in samples])) for k in samples[0] if k not in ("V", "Vc")}
    fs = V_fine / samples[0]["V"]
    cs = Vc / samples[0]["Vc"]
    st = tuned_stats
    outer = outer_per_col
    waves = ncol // 8
    n_cycles = st["n_bottom_solves"] / waves
    bottom = st["avg_bottom_iters"]
    # per column: every outer step = fine operator (FGMRES) + cycle (restrict,
    # bottom GMRES, prolong, fine residual, SAP) + an outer Gram-Schmidt step;
    # every bottom step = coarse operator + Gram-Schmidt step
    per_cycle = (m["restrict"] + m["prolong"] + m["fine_op"] + m["sap"]) * fs + bottom * (
        m["coarse_op"] + m["gram_coarse"]) * cs
    per_outer = m["fine_op"] * fs + m["gram_fine"] * fs
    per_col = n_cycles * per_cycle + outer * per_outer
    c1 = raw["c1"]
    return dict(value=cores / per_col, unit="rhs*shift solves/s", cores=cores, kind="oracle",
                cpu_model=raw["cpu_model"], nproc=os.cpu_count(),
                sample=(f"FP64 numpy oracle, one column per process on {cores} processes at once (one thread "
                        f"each): per-operation timings of the two-level method on 8x8x8x16 sub-lattices drawn "
                        f"with the 40^3x80 recipe ({raw['c5_wall']:.0f}s wall), scaled per site to 40x40x40x80 "
                        f"and multiplied by the GPU solve's counts per column ({n_cycles:.0f} cycles of "
                        f"{bottom:.1f} coarse GMRES steps, {outer:.1f} outer steps): {per_col:.0f}s per column; "
                        f"extrapolated, not a full solve"),
                c1_full_solves={"columns": 6, "wall_s": raw["c1_wall"], "solves_per_s": 6 / raw["c1_wall"],
                                "processes": min(cores, 6), "all_converged": all(ok for _, ok in c1),
                                "seconds_per_column": [round(t, 2) for t, _ in c1],
                                "workload": "tm_4x4x4x4_2rhs_3shift (4^4, kappa 0.14, two-level MG), full "
                                            "oracle solves to 1e-10"},
                per_op_seconds_per_site={k: v / (samples[0]["Vc"] if k in ("coarse_op", "gram_coarse")
                                                 else samples[0]["V"]) for k, v in m.items()})


# --------------------------------------------------------------- learned study ---
# Learned-smoother study: 16^3x32 fields drawn like the 16^3x32 workload's
# (eps 0.3, kappa 0.150), 8 training and 4 held-out gauge seeds; 8 x 160 Adam
# steps of 16 residual -> error pairs (20480 pairs), errors from 0..2 SAP
# sweeps; the trained net (4 minimal-residual steps per call, SAP fallback)
# replaces SAP in FGMRES(40) on 3 rhs x 4 shifts per held-out field.
LEARNED_TRAIN_SEEDS = tuple(range(4101, 4109))
LEARNED_HELDOUT_SEEDS = tuple(range(4201, 4205))
LEARNED = dict(steps=160, batch=16, lr=2e-3, sap_sweeps=2, cycles=4, n_rhs=3)
LEARNED_SOLVER = dict(n_levels=1, sap_cycles=1, sap_mr_iters=12, outer_restart=40, max_outer=3000)


def learned_study(dd, S, np, torch):
    w = S.workload(SMALL)
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
        c = dd.Context(dd.params_for_workload(w, precision=dd.MIXED, **{**LEARNED_SOLVER, **kw}), U)
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


# --------------------------------------------------------------- main ---
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed solves of one right-hand side (8 columns, one wave) before the timed steps")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-three", action="store_true", help="skip the three-level hierarchy on 40^3x80")
    ap.add_argument("--no-small", action="store_true", help="skip the 16^3x32 forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ab", action="store_true", help="skip the plain one-wave solves with the one- and two-reduction Gram step")
    ap.add_argument("--learned", action="store_true",
                    help="instead of the solve benchmark, train the learned smoother on 8 gauge fields and "
                         "compare it with SAP on 4 held-out fields")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (it would shard by 4-d "
              "domain decomposition with halo exchanges, which is not built); run it with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    raw_cpu = None
    if not args.no_cpu_baseline and not args.learned:
        log("cpu baseline: oracle on the host cores (before the GPU is touched)")
        raw_cpu = cpu_measure()

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
    wu = 1 if args.warmup else 0

    # tuned form, with live HIP-event timing of the roofline kernel class
    ctx, tuned = run_form(dd, torch, w, U, b, mus, dd.MIXED, TUNED, args.steps, wu, 8, ROOFLINE_CLASS, "tuned")
    value = tuned["solves_per_s"]
    st = tuned["stats"]
    # fine stencil bandwidth on this lattice (one wave of 8 columns, HIP events)
    V = w.volume
    n_iter = 10
    t32 = ctx.time_op(0, 0, dd.FP32, 8, n_iter)
    t64 = ctx.time_op(0, 0, dd.FP64, 8, n_iter)
    links32 = 288 if tuned["tuned"]["fp32_links"] == 0 else 192
    bytes32 = V * (links32 + 8 * 48 * 4)
    bytes64 = V * (576 + 8 * 48 * 8)
    Vc, dc, _ = ctx.level_info(1)
    # plain copy kernel of one FP64 8-column vector (read + write), the
    # reference for the bandwidth and for calibrating the traffic counters
    t_copy = ctx.time_op(5, 0, dd.FP64, 8, 5)
    copy_bytes = 2 * V * 12 * 16 * 8
    tuned.pop("x")
    # the level-1 coarse stencil, timed live in one more (untimed) solve of
    # one wave (1 rhs x 8 shifts)
    ctx.set_tuning("time_kernel", TIMED["coarse1"])
    ctx.solve(mus, b[:1].contiguous())
    st_c = ctx.stats()
    ctx.set_tuning("time_kernel", 0)
    ctx.close()
    torch.cuda.empty_cache()

    # roofline of the dominant kernel: the FP32 odd-even SAP half sweep, bound
    # by its arithmetic issue (the counter summary in profiles/), against the
    # published FP32 vector peak
    n_l, ms_l, tiles_l = st["n_sap_kernels"], st["sap_kernel_ms"], st["n_sap_kernel_tiles"]
    k_mr = TUNED["sap_mr_iters"]
    flops_tile = sap_oe_flops_per_tile(V, k_mr)
    achieved = tiles_l * flops_tile / (ms_l * 1e-3) / 1e12 if n_l else None
    roofline = {"kernel": f"k_sap_oe<float, 2, float, 2> (FP32 odd-even SAP half sweep, {k_mr} MR steps, one "
                          "8-column tile per launch)",
                "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS if achieved else None, "traffic": counter_traffic(SAP_PROFILE, SAP_SRC),
                "traffic_source": "profiles/k_sap_oe_fp32_40x40x40x80_8col.md (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 "
                                  "per launch, factors from the copy kernel)",
                "us_per_launch": ms_l * 1e3 / n_l if n_l else None, "launches_timed": n_l,
                "timed_in": "the timed solves", "algorithmic_flops_per_launch": tiles_l * flops_tile / n_l if n_l else None,
                "frac_of_unpacked_fp32": achieved / (FP32_PEAK_TFLOPS / 2) if achieved else None}
    # the level-1 coarse stencil on BF16 MFMA, HBM bound (its blocks, 1.7 GB,
    # stream from HBM at every launch)
    n_c, ms_c, tiles_c = st_c["n_sap_kernels"], st_c["sap_kernel_ms"], st_c["n_sap_kernel_tiles"]
    bytes_tile, cflops_tile = coarse1_bytes_flops(Vc, dc, 1)
    blocks_bytes = Vc * 9 * 4 * dc * dc
    alg_bytes = n_c * blocks_bytes + tiles_c * (bytes_tile - blocks_bytes)
    c_ach = alg_bytes / (ms_c * 1e-3) / 1e9 if n_c else None
    roofline_coarse = {"kernel": "k_coarse_mfma_t1<48, _Float16> (level-1 coarse stencil on the FP16 basis vector, "
                                 "BF16 MFMA, FP32 accumulation)",
                       "bound": "hbm", "achieved": c_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": c_ach / HBM_PEAK_GBS if c_ach else None, "traffic": counter_traffic(),
                       "traffic_source": "profiles/k_coarse_mfma_t1_48_40x40x40x80_8col.md",
                       "us_per_launch": ms_c * 1e3 / n_c if n_c else None, "launches_timed": n_c,
                       "timed_in": "one untimed solve of one wave after the timed steps",
                       "algorithmic_bytes_per_launch": alg_bytes / n_c if n_c else None,
                       "mfma_TFLOPs": (n_c and tiles_c * cflops_tile / (ms_c * 1e-3) / 1e12)}

    plain = None
    gram_ab = None
    if not args.no_plain:
        pctx, plain = run_form(dd, torch, w, U, b, mus, dd.PLAIN_FP64, PLAIN, args.steps, wu, 8, None, "plain")
        plain.pop("x")
        # one wave (1 rhs x 8 shifts) of the plain form, whose outer and
        # coarse Krylov bases are FP64, with the one- and the two-reduction
        # Gram-Schmidt step (dots, update with norm, normalisation pass)
        if not args.no_ab:
            b1 = b[:1].contiguous()
            gram_ab = {}
            for knob, key in ((1, "one_reduction_seconds"), (0, "two_reduction_seconds")):
                pctx.set_tuning("gram_one_reduction", knob)
                torch.cuda.synchronize()
                t0 = time.time()
                _, inf2, _ = pctx.solve(mus, b1)
                torch.cuda.synchronize()
                gram_ab[key] = time.time() - t0
                gram_ab[key.replace("seconds", "all_converged")] = all(i["converged"] for i in inf2)
            pctx.set_tuning("gram_one_reduction", 1)
            gram_ab["form"] = "plain FP64 two-level, one wave of 8 columns"
            log(f"  plain one wave, one / two reductions: {gram_ab['one_reduction_seconds']:.2f}s / "
                f"{gram_ab['two_reduction_seconds']:.2f}s")
        pctx.close()
        torch.cuda.empty_cache()
    three = None
    if not args.no_three:
        # one wave (1 rhs x 8 shifts): the three-level hierarchy, and its
        # coarsest GMRES restarted every 10 steps without and with deflation
        three = {}
        for name, form in (("bottom_gmres63", THREE), ("bottom_gmres10", THREE_R10),
                           ("bottom_gmres_dr10_4", THREE_DR)):
            tctx, r = run_form(dd, torch, w, U, b[:1].contiguous(), mus, dd.MIXED, form, 1, 1, 8, None,
                               "three-level " + name)
            r.pop("x")
            tctx.close()
            torch.cuda.empty_cache()
            three[name] = summary(r, "f64 outer / f32 cycle")

    small = None
    if not args.no_small:
        ws = S.workload(SMALL)
        Us = S.gauge_field(ws.dims, ws.eps, ws.seed_gauge)
        bs = torch.from_numpy(S.rhs_for(ws)).cuda()
        ms = np.array(ws.mus)
        small = {}
        for name, prec, solver in (("one_level", dd.MIXED, SMALL_ONE), ("two_level", dd.MIXED, SMALL_TWO),
                                   ("three_level", dd.MIXED, SMALL_THREE),
                                   ("two_level_plain_fp64", dd.PLAIN_FP64, SMALL_TWO)):
            c, r = run_form(dd, torch, ws, Us, bs, ms, prec, solver, 1, 12, ws.n_col, None, "16^3x32 " + name)
            r.pop("x")
            c.close()
            small[name] = summary(r, "f64" if prec == dd.PLAIN_FP64 else "f64 outer / f32 cycle")
        # the paper's "old" mode: the plain FP64 two-level solver taking one
        # column (one rhs, one shift) at a time, on the 8 columns of the first
        # two right-hand sides (the batched forms above take all 48 at once)
        c, r = run_form(dd, torch, ws, Us, bs[:2].contiguous(), ms, dd.PLAIN_FP64, dict(SMALL_TWO, max_active_cols=1),
                        1, 1, ws.n_col, None, "16^3x32 two_level_plain_fp64_one_column_at_a_time")
        r.pop("x")
        c.close()
        small["two_level_plain_fp64_one_column_at_a_time"] = summary(r, "f64")
        # non-degenerate doublets on the same lattice and hierarchy: the 12 Z2
        # fields as 6 flavour doublets, mubar = 0.12, epsbar = 0.11, FP64
        # FGMRES over the flavour-diagonal two-level cycle
        p = dd.params_for_workload(ws, precision=dd.MIXED, **SMALL_TWO)
        c = dd.Context(p, Us)
        c.autotune(ws.n_col)
        bnd = bs.reshape(6, 2, *bs.shape[1:]).contiguous()
        mub, epb = np.full(6, 0.12), np.full(6, 0.11)
        c.solve_nd(mub, epb, bnd)
        torch.cuda.synchronize()
        t0 = time.time()
        xnd, inf_nd, st_nd = c.solve_nd(mub, epb, bnd)
        torch.cuda.synchronize()
        el = time.time() - t0
        small["nd_two_level"] = {"doublets_per_s": 6 / el if st_nd == dd.OK else 0.0, "seconds": el,
                                 "all_converged": st_nd == dd.OK,
                                 "worst_err_vs_fp64": max(i["err_vs_fp64"] for i in inf_nd),
                                 "outer_iters_max": max(i["outer_iters"] for i in inf_nd),
                                 "mubar": 0.12, "epsbar": 0.11, "doublets": 6}
        c.close()
        log(f"  16^3x32 doublets: {el:.2f}s, {small['nd_two_level']}")
        small["config"] = {"workload": ws.name, "lattice": "16x16x16x32", "kappa": ws.kappa, "columns": ws.n_col,
                           "one_level": "FP64 FGMRES(4) over FP32 FGMRES(40, FP16 basis) over SAP",
                           "two_level": "FP64 FGMRES(40) over the two-level cycle (4^4 aggregates, N = 24)",
                           "three_level": "FP64 FGMRES(40) over the three-level cycle (4^4 then 2^4, N = 24 / 32)",
                           "two_level_plain_fp64_one_column_at_a_time": "the plain FP64 two-level form with one "
                           "column in flight (no batching of rhs and shifts), 8 columns"}

    # the oracle runs the plain method (FP64 FGMRES over the cycle): its
    # counts per column are the plain GPU form's (the tuned form's if the
    # plain one was skipped, its inner steps counted as outer ones)
    if plain:
        cnt, outer_col = plain["stats"], plain["outer_iters_mean"]
    else:
        cnt, outer_col = st, tuned["outer_iters_mean"] + st["n_inner_iters"] / (ncol // 8)
    cpu = cpu_baseline(raw_cpu, cnt, outer_col, ncol, V, Vc) if raw_cpu else None

    out = {
        "metric": "rhs*shift solves/s at true FP64 relative residual 1e-10 (tuned form); dslash HBM GB/s",
        "value": value,
        "unit": "rhs*shift solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tuned["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 cycle / bf16 coarse blocks",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": "40x40x40x80", "kappa": w.kappa, "eps": w.eps, "n_rhs": w.n_rhs,
                   "shifts": list(w.mus), "columns": ncol, "tol": 1e-10, "columns_in_flight": 8,
                   "solver": "FP64 FGMRES(1) over FP32 FGMRES(12, FP16 basis) to 1e-2 over the two-level "
                             "aggregation MG cycle in FP32 (4^4 aggregates, N = 24, two setup rounds and two "
                             "bootstrap rounds, FP16 P in the transfers; red-black SAP 1 cycle of 5 MR steps on "
                             "the odd-even reduced 4^4 blocks; coarse GMRES on gamma5_c D_c to 0.15 with an FP16 "
                             "basis, BF16 MFMA stencil)",
                   "plain_solver": "FP64 FGMRES(4) over the same two-level hierarchy and cycle, every step in "
                                   "FP64"},
        "all_converged": tuned["allconv"],
        "worst_true_rel_res": tuned["worst"],
        "tuned": summary(tuned, "f64 outer / f32 cycle / bf16 coarse blocks"),
        "plain_fp64": summary(plain, "f64") if plain else None,
        "tuned_over_plain": (value / plain["solves_per_s"]) if plain and plain["solves_per_s"] else None,
        "three_level_one_wave": three,
        "autotuned": tuned["tuned"],
        "gram_one_vs_two_reductions": gram_ab,
        "dslash_40x40x40x80_8col": {"fp32_us": t32 * 1e6, "fp32_GBs": bytes32 / t32 / 1e9,
                                    "fp32_GFLOPs": 1320 * V * 8 / t32 / 1e9,
                                    "fp64_us": t64 * 1e6, "fp64_GBs": bytes64 / t64 / 1e9,
                                    "fp64_GFLOPs": 1320 * V * 8 / t64 / 1e9,
                                    "fp32_hbm_frac": bytes32 / t32 / 1e9 / HBM_PEAK_GBS,
                                    "fp64_hbm_frac": bytes64 / t64 / 1e9 / HBM_PEAK_GBS},
        "roofline": roofline,
        "roofline_coarse_stencil": roofline_coarse,
        "copy_kernel_GBs": copy_bytes / t_copy / 1e9,
        "small_16x16x16x32": small,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
