"""Benchmark: sigma-builds/s and time-to-roots of the full DF-SS-FNO-EA-ADC(3) solve on one MI355X.

One step = one call of adc3_ea_solve on the named workload (default: o=20, v=200,
X=600, seed 1, 5 roots, SS-FNO threshold 10^-4.5, NAF threshold 1e-2, Davidson
conv 1e-6 Eh, perturbative correction on): canonical MP2 + EA-ADC(2), then per
root D^SS, natural orbitals, recanonicalisation, NAF, EA-ADC(2) and EA-ADC(3) in
the truncated basis and the correction.  Inputs are resident in HBM before the
timed region.

value  = sigma vectors built during the timed solves / timed wall time
ms_per_step = time to all roots (one full solve)

Usage: python bench.py [--steps K] [--warmup W] [--workload NAME] [--scale s]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0
# worker slots of the batched study: three slices of the largest instance's plan (193 GB of workspace) fit
# in HBM beside the inputs; measured with worker threads: 1 slot 47.6 s, 2 slots 36.3 s, 3 slots 31.7 s
BATCH_SLOTS = 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ssfno-o20v200x600")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32/BF16 mixed-precision solves")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner study")
    ap.add_argument("--no-large-form", action="store_true",
                    help="skip the large workload's form: its assembled ladder at full shape in FP64 / FP32 / BF16, "
                         "and a scaled-down instance solved in the three precisions against the oracle's golden")
    ap.add_argument("--learned-full", action="store_true",
                    help="also compare the learned preconditioner with Jacobi at o=30 v=400 X=1200 (251 GB)")
    ap.add_argument("--batched", type=int, default=64,
                    help="also solve the first N instances of the ragged batched workload (seeds 100..; 0 = skip)")
    ap.add_argument("--batched-lockstep-only", action="store_true",
                    help="batched workload: the lockstep engine only (default: worker threads with a cold "
                         "tuner, then lockstep and worker threads again with the tuner settled)")
    ap.add_argument("--no-lockstep", action="store_true",
                    help="skip the comparison solves of the headline workload with one basis at a time and "
                         "with the lockstep engine (the timed steps use the library's default, the per-root "
                         "bases each on a host thread and stream of its own)")
    ap.add_argument("--large-mixed", type=float, default=0.0,
                    help="also run the FP64 / FP32 / BF16 Davidson study of the o=40 v=600 X=1800 workload "
                         "with B scaled by this factor (about 12 minutes; 0 = skip)")
    ap.add_argument("--large-mixed-precs", default="0,1,2",
                    help="Davidson precisions of the large study (0 FP64, 1 FP32, 2 BF16), comma-separated")
    ap.add_argument("--large-mixed-ref", default="",
                    help="FP64 roots of the large study from an earlier run (comma-separated), when 0 is not run")
    ap.add_argument("--sigma-reps", type=int, default=10)
    ap.add_argument("--sigma-only", action="store_true",
                    help="profiling mode: only the isolated ADC(3) sigma builds plus a 2 GiB copy (counter calibration)")
    ap.add_argument("--sigma-precision", type=int, default=0,
                    help="precision of the --sigma-only context and its sigma calls (0 FP64, 1 FP32, 2 BF16 ladder)")
    ap.add_argument("--dfladder-only", action="store_true",
                    help="profiling mode: the assembled ladder alone at o=40 v=600 X=1800 (5 vectors) in FP64, FP32 "
                         "and BF16, plus a 2 GiB copy (counter calibration)")
    ap.add_argument("--dfladder-precs", default="0,1,2",
                    help="operand precisions of --dfladder-only (0 FP64, 1 FP32, 2 BF16)")
    ap.add_argument("--variant-scale", type=float, default=0.018,
                    help="also time one solve with B scaled by this factor (weak correlation, FNO truncates); 0 = skip")
    return ap.parse_args()


# HBM traffic of the ladder kernel per launch, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) of `bench.py --sigma-only`, each scaled by the same counter's reading
# for a copy of known size.  Keyed by a hash of the kernel's source and of the pair-block packing
# that sets its launch shapes: a change to either reports null until it is measured again.
LADDER_TRAFFIC = {
    "25bbecc6313e593a": {
        "bytes_per_launch": 3.436e9, "read_bytes": 3.307e9, "written_bytes": 0.129e9,
        "fetch_scale": 2.0, "write_scale": 1.0,
        "measured_on": "sigma ladder o=20 v=200 X=128, 5 vectors (M=100, ladder_f64t_kernel), 8 K-chunks (fixed "
                       "with ADC3_LADDER_CHUNKS=8; the tuner takes 8 or 16, and 16 adds 0.13 GB of partial sums to a "
                       "launch); mean of the pair-symmetric (3.478 GB) and pair-antisymmetric (3.394 GB) block launches",
        "profile": "profiles/ladder_f64t_o20v200x128_sigma_counters.md"},
}


def oracle_golden(name):
    """Roots the FP64 oracle stored for a workload (tests/golden, written by make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def vs_oracle(np, roots, gold):
    """max |omega - omega_oracle| over the roots the golden holds (None without a golden)."""
    if gold is None:
        return None
    ref = np.array(gold["roots"], dtype=float)
    k = min(len(ref), len(roots))
    return float(np.abs(np.asarray(roots, dtype=float)[:k] - ref[:k]).max())


def golden_name(workload, scale):
    return workload if scale == 1.0 else "%s_s%s" % (workload, repr(scale))


def stored_pair_elems(v):
    """Elements of the stored ladder's pair blocks (c <= d and c < d sides, each padded to a multiple of 8)."""
    lp = (v * (v + 1) // 2 + 7) // 8 * 8
    lm = (v * (v - 1) // 2 + 7) // 8 * 8
    return lp * lp + lm * lm


def min_factor(X, v, o, nv_max=16):
    """F_lad,min / executed flops of a stored-ladder block of n_v vectors, executed = 2 o n_v (lp^2 + lm^2)
    (the two pair blocks, about o v^4 n_v), F_lad,min = min(4 X o v^3 n_v (assembled from the factor),
    executed); the smaller ratio over n_v = 1..nv_max, so the figure is never overstated."""
    ex = [2.0 * o * n * stored_pair_elems(v) for n in range(1, nv_max + 1)]
    r = [min(4.0 * X * o * v ** 3 * n, e) / e for n, e in zip(range(1, nv_max + 1), ex)]
    return min(r)


def ladder_traffic():
    """The ladder kernel's source and the pair-block packing that sets its launch shapes, hashed together."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_05897_amd", "csrc")
    h = hashlib.sha256()
    for f in ("ladder.hip", "ladder_sa.hip"):
        h.update(open(os.path.join(d, f), "rb").read())
    h = h.hexdigest()[:16]
    return h, LADDER_TRAFFIC.get(h)


def learned_study(adc, d, torch, np):
    """Learned preconditioner vs Jacobi (ADC(3), 5 roots, conv 1e-6, scale 0.3): for each shape,
    collect 2000 groups from Jacobi solves of seeds 200-239, train on the GPU, then solve the
    held-out seeds 240-243 both ways (iterations, wall time, root agreement)."""
    import synth
    scale, nroots, out = 0.3, 5, {}
    for shape in ((6, 40, 120), (16, 120, 360)):
        t0 = time.perf_counter()
        Fs, As, Ds = [], [], []
        for seed in range(200, 240):
            eo, ev, B = synth.make_instance(*shape, seed, scale=scale)
            ctx = adc.Context(d(eo), d(ev), d(B), 3, nroots=nroots)
            F, A, D, _ = ctx.mlp_collect(nroots, 1e-6, 256, 50, seed)
            Fs.append(F)
            As.append(A)
            Ds.append(D)
            ctx.close()
        F, A, D = torch.cat(Fs), torch.cat(As), torch.cat(Ds)
        t_collect = time.perf_counter() - t0
        w = torch.as_tensor(synth.mlp_init(1), device="cuda")
        t0 = time.perf_counter()
        losses = adc.adc3_mlp_train(w, F, A, D, epochs=60, batch_groups=32, lr=2e-3, seed=7)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        print("learned: o%dv%dx%d collected in %.1f s, trained in %.1f s" % (*shape, t_collect, t_train),
              file=sys.stderr, flush=True)
        held = {"jacobi": {"iterations": 0, "wall_s": 0.0}, "learned": {"iterations": 0, "wall_s": 0.0}}
        dmax, statuses = 0.0, []
        for seed in range(240, 244):
            eo, ev, B = synth.make_instance(*shape, seed, scale=scale)
            ctx = adc.Context(d(eo), d(ev), d(B), 3, nroots=nroots)
            ctx.davidson(nroots, 1e-6)  # warm-up (tuner, first launches)
            roots = {}
            for tag, weights in (("jacobi", None), ("learned", w)):
                ctx.set_preconditioner(weights)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                wr, _, _, it, st = ctx.davidson(nroots, 1e-6)
                torch.cuda.synchronize()
                held[tag]["iterations"] += it
                held[tag]["wall_s"] += time.perf_counter() - t1
                roots[tag] = wr
                statuses.append(st)
            dmax = max(dmax, float(np.abs(roots["learned"] - roots["jacobi"]).max()))
            ctx.close()
        out["o%dv%dx%d" % shape] = {
            "train": {"seeds": "200-239", "groups": int(F.shape[0]), "group_size": 256, "collect_s": t_collect,
                      "train_s": t_train, "epochs": 60, "loss_first_last": [float(losses[0]), float(losses[-1])]},
            "held_out": {"seeds": "240-243", **held, "statuses": statuses,
                         "iteration_ratio": held["learned"]["iterations"] / max(held["jacobi"]["iterations"], 1),
                         "wall_ratio": held["learned"]["wall_s"] / held["jacobi"]["wall_s"],
                         "max_abs_root_diff_Eh": dmax}}
        print("learned: o%dv%dx%d held-out solves done" % shape, file=sys.stderr, flush=True)
    return {"scale": scale, "level": 3, "nroots": nroots, "conv": 1e-6, "shapes": out}


def batched_study(adc, d, torch, np, n, modes=((0, "threads_cold_tuner"), (1, "lockstep"), (0, "threads"))):
    """The ragged batched workload: instances of seeds 100.. (nocc~U{5..30}, nvir~U{50..300},
    naux = 3 nvir, literal scale), 8 roots, conv 1e-6, FP32 ladder, BATCH_SLOTS worker slots.  Engine 1:
    the lockstep block Davidson (waves of one instance per slot, chunks of iterations replayed from graphs
    on each instance's stream, device-side convergence flags); engine 0: one host thread per worker
    stream, sigma passes replayed from graphs.  The first run of a process also pays the ladder tuner's trial launches for every new
    shape (about 64 x 2 x 2 of them), so the engines are compared on later runs.  Instance generation is
    not timed."""
    import synth
    inst = []
    g0 = time.perf_counter()
    for s in range(100, 100 + n):
        eo, ev, B = synth.batch_instance(s)
        inst.append(dict(eps_occ=d(eo), eps_vir=d(ev), B=d(B), nroots=8, conv=1e-6))
        del B
    gen_s = time.perf_counter() - g0
    print("batched: %d instances generated in %.1f s" % (n, gen_s), file=sys.stderr, flush=True)
    sum_n = sum(int(x["eps_vir"].numel()) * (1 + int(x["eps_occ"].numel()) * int(x["eps_vir"].numel())) for x in inst)
    out = {"instances": n, "seeds": "100-%d" % (99 + n), "nroots": 8, "conv": 1e-6, "precision": "fp32 ladder",
           "slots": BATCH_SLOTS, "sum_N": sum_n, "generation_s_untimed": gen_s}
    ref = None
    for mode, label in modes:
        o = adc.adc3_default_opts()
        o.precision = 1
        o.sigma_graphs = 1
        o.lockstep = mode
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            nbytes = adc.adc3_ea_solve_batched_workspace_bytes(inst, o, BATCH_SLOTS)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            roots, reps, sts, st = adc.adc3_ea_solve_batched(inst, o, BATCH_SLOTS, workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        sig = sum(rr[0]["sigma_builds"] for rr in reps)  # each instance's count sits on its root 0
        res = {"time_s": dt, "workspace_GB": nbytes / 1e9, "status": st, "statuses": [int(x) for x in sts],
               "statuses_ok": sum(1 for x in sts if x == 0), "sigma_builds": sig, "sigma_builds_per_s": sig / dt,
               "iterations": [rr[0]["iters"] for rr in reps],
               "max_resnorm": float(max(r["resnorm"] for rr in reps for r in rr))}
        golds = [(i, oracle_golden("batch-seed%d" % (100 + i))) for i in range(n)]
        golds = [(i, g) for i, g in golds if g is not None]
        if golds:
            res["oracle_goldens"] = {"seeds": [100 + i for i, _ in golds],
                                     "max_abs_root_diff_Eh": max(vs_oracle(np, roots[i], g) for i, g in golds)}
        if ref is None:
            ref = roots
        else:
            res["max_rel_root_diff_vs_first_run"] = float(max(
                np.abs(a - b).max() / max(1.0, np.abs(a).max()) for a, b in zip(ref, roots)))
        out[label] = res
        print("batched: %s %.1f s, %d of %d converged" % (label, dt, res["statuses_ok"], n), file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    return out


def learned_full_size(adc, d, torch, np, scale, train_seeds=range(200, 206), eval_seeds=(240, 241)):
    """The learned preconditioner at its own workload's shape: o=30, v=400, X=1200, scale 0.3, 5 roots,
    conv 1e-6, the ladder stored as its pair blocks (102 GB).  Training data from Jacobi solves of
    `train_seeds` (fewer than the workload's 40 seeds 200-239: each solve here takes seconds), GPU
    training, then Jacobi and learned solves of the held-out `eval_seeds` (iterations, wall time, roots)."""
    import synth
    shape, nroots, conv = (30, 400, 1200), 5, 1e-6
    Fs, As, Ds = [], [], []
    t0 = time.perf_counter()
    for seed in train_seeds:
        eo, ev, B = synth.make_instance(*shape, seed, scale=scale)
        ctx = adc.Context(d(eo), d(ev), d(B), 3, nroots=nroots, ladder=1)
        del B
        F, A, D, _ = ctx.mlp_collect(nroots, conv, 256, 50, seed)
        Fs.append(F)
        As.append(A)
        Ds.append(D)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        print("learned-full: collected seed %d" % seed, file=sys.stderr, flush=True)
    t_collect = time.perf_counter() - t0
    w = torch.as_tensor(synth.mlp_init(1), device="cuda")
    t0 = time.perf_counter()
    F, A, D = torch.cat(Fs), torch.cat(As), torch.cat(Ds)
    losses = adc.adc3_mlp_train(w, F, A, D, epochs=60, batch_groups=32, lr=2e-3, seed=7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    out = {"shape": list(shape), "scale": scale, "nroots": nroots, "conv": conv, "ladder": "stored pair blocks",
           "train_seeds": [int(x) for x in train_seeds], "groups": int(F.shape[0]), "collect_s": t_collect,
           "train_s": t_train, "loss_first_last": [float(losses[0]), float(losses[-1])], "eval": {}}
    del Fs, As, Ds, F, A, D
    tot = {"jacobi": [0, 0.0], "learned": [0, 0.0]}
    for seed in eval_seeds:
        eo, ev, B = synth.make_instance(*shape, seed, scale=scale)
        ctx = adc.Context(d(eo), d(ev), d(B), 3, nroots=nroots, ladder=1)
        del B
        ctx.davidson(nroots, conv)  # warm-up: the ladder tuner settles every row count the solve meets
        res = {}
        for tag, weights in (("learned", w), ("jacobi", None)):
            ctx.set_preconditioner(weights)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            wr, _, rn, it, st = ctx.davidson(nroots, conv)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            res[tag] = {"iterations": it, "wall_s": dt, "status": st, "roots": [float(x) for x in wr]}
            tot[tag][0] += it
            tot[tag][1] += dt
            print("learned-full: seed %d %s %d iterations %.2f s" % (seed, tag, it, dt), file=sys.stderr, flush=True)
        res["max_abs_root_diff_Eh"] = float(np.abs(np.array(res["learned"]["roots"]) -
                                                   np.array(res["jacobi"]["roots"])).max())
        out["eval"][str(seed)] = res
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    out["iterations_learned_vs_jacobi"] = [tot["learned"][0], tot["jacobi"][0]]
    out["wall_s_learned_vs_jacobi"] = [tot["learned"][1], tot["jacobi"][1]]
    out["wall_ratio"] = tot["learned"][1] / tot["jacobi"][1]
    return out


def mixed_ladder_dominated(adc, d, torch, np):
    """ADC(3) Davidson (5 roots, conv 1e-6) on o=20, v=300, X=900, seed 3, scale 0.3 -- a shape where the
    ladder dominates each iteration -- with FP64, FP32-ladder and BF16-ladder sigma (the reduced
    phases end with an FP64 restart).  Context setup (FP64 in every mode) is not timed."""
    import synth
    eo, ev, B = synth.make_instance(20, 300, 900, 3, scale=0.3)
    tB = d(B)
    del B
    out, ref = {}, None
    for prec, tag in ((0, "fp64"), (1, "fp32"), (2, "bf16")):
        ctx = adc.Context(d(eo), d(ev), tB, 3, nroots=5, precision=prec)
        ctx.davidson(5, 1e-6, precision=prec)  # warm-up: tuner, first launches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, _, rn, it, st = ctx.davidson(5, 1e-6, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if ref is None:
            ref = w
        out[tag] = {"davidson_s": dt, "iterations": it, "status": st,
                    "max_abs_root_diff_vs_fp64_Eh": float(np.abs(w - ref).max())}
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    out["shape"] = [20, 300, 900]
    out["roots_fp64"] = [float(x) for x in ref]
    for tag in ("fp32", "bf16"):
        out[tag]["speedup_vs_fp64"] = out["fp64"]["davidson_s"] / out[tag]["davidson_s"]
    return out


def large_mixed_study(adc, d, torch, np, scale, precs=(0, 1, 2), ref=None):
    """ADC(3) Davidson of the large mixed-precision workload (o=40, v=600, X=1800, seed 2, canonical basis,
    5 roots, conv 1e-6), B scaled by `scale`, with FP64, FP32-operand and BF16-operand sigma (each
    reduced-precision Davidson ends with an FP64 restart).  The ladder is assembled from the DF factor in
    every application (its stored pair blocks would take 518 GB).  Context setup (FP64 in every mode) is
    timed on its own; the FP64 run shares the first reduced-precision context.  `ref`: FP64 roots of an
    earlier run when 0 is not in `precs`."""
    import synth
    p, eo, ev, B = synth.preset("mixed-o40v600x1800", scale=scale)
    tB = d(B)
    del B
    nroots, conv = p["nroots"], p["conv"]
    out = {"shape": [p["nocc"], p["nvir"], p["naux"]], "seed": p["seed"], "scale": scale, "nroots": nroots,
           "conv": conv, "ladder": "assembled from the DF factor"}
    if ref is not None:
        ref = np.asarray(ref, dtype=float)
        out["fp64_roots_from_earlier_run"] = [float(x) for x in ref]
    groups = []
    lp = [x for x in (1, 2) if x in precs]
    for i, cp in enumerate(lp):
        groups.append((cp, ((0,) if (0 in precs and i == 0) else ()) + (cp,)))
    if not lp and 0 in precs:
        groups.append((0, (0,)))
    for cprec, runs in groups:
        t0 = time.perf_counter()
        ctx = adc.Context(d(eo), d(ev), tB, 3, nroots=nroots, precision=cprec)
        torch.cuda.synchronize()
        out["setup_s_precision%d_context" % cprec] = time.perf_counter() - t0
        print("large mixed: context (precision %d) built" % cprec, file=sys.stderr, flush=True)
        for pr in runs:
            tag = ("fp64", "fp32", "bf16")[pr]
            kind = adc.PROF_LADDER if pr == 0 else adc.PROF_LADDER_LP
            adc.adc3_profile_enable(True)
            t1 = time.perf_counter()
            w, _, rn, it, st = ctx.davidson(nroots, conv, precision=pr)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            lms, ln, lf, lb = adc.adc3_profile_query(kind)
            lbound = adc.adc3_profile_query_bound(kind)
            sig_ms, _, _, _ = adc.adc3_profile_query(adc.PROF_SIGMA)
            adc.adc3_profile_enable(False)
            if ref is None:
                ref = w
            peak = (78.6, 157.3, 2500.0)[pr]
            ach = lf / (lms * 1e-3) / 1e12 if lms > 0 else 0.0
            out[tag] = {"davidson_s": dt, "iterations": it, "status": st, "roots": [float(x) for x in w],
                        "max_resnorm": float(np.max(rn)),
                        "root_diff_vs_fp64_Eh": [float(x) for x in (w - ref)],
                        "sigma_ms": sig_ms,
                        "ladder": {"launches": ln, "total_ms": lms, "achieved_tflops": ach, "peak_tflops": peak,
                                   "frac": ach / peak, "bound_time_frac": lbound / lms if lms > 0 else None}}
            print("large mixed: %s Davidson %.1f s, %d iterations" % (tag, dt, it), file=sys.stderr, flush=True)
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    for tag in ("fp32", "bf16"):
        if tag in out and "fp64" in out:
            out[tag]["speedup_vs_fp64"] = out["fp64"]["davidson_s"] / out[tag]["davidson_s"]
    return out


def large_workload_form(adc, d, torch, np):
    """The large mixed-precision workload's path, within the default run's time: (1) its dominant sigma term,
    the ladder assembled from the DF factor, at the full shape (v = 600, X = 1800, 200 rows) in FP64, FP32 and
    BF16 operands (one untimed and one timed call each); (2) a scaled-down instance of the same form (o=16,
    v=160, X=480, seed 2, B x 0.05, 5 canonical roots, the ladder assembled in every application) solved
    with FP64, FP32 and BF16 sigma (reduced phases ending with the FP64 restart), each after one untimed
    solve, against the FP64 oracle's stored roots (conv 1e-9)."""
    import synth
    out = {"ladder_full_shape": dfladder_only(adc, torch, 1)}
    g = oracle_golden("large-like-o16v160x480_s0.05")
    eo, ev, B = synth.make_instance(g["nocc"], g["nvir"], g["naux"], g["seed"], scale=g["scale"])
    teo, tev, tB = d(eo), d(ev), d(B)
    inst = {"nocc": g["nocc"], "nvir": g["nvir"], "naux": g["naux"], "seed": g["seed"], "scale": g["scale"],
            "nroots": 5, "conv": 1e-7, "ladder": "assembled"}
    ref = None
    for prec, tag in ((0, "fp64"), (1, "fp32"), (2, "bf16")):
        o = adc.adc3_default_opts()
        o.ladder, o.precision = 2, prec
        ws = torch.empty(adc.adc3_ea_solve_workspace_bytes(g["nocc"], g["nvir"], g["naux"], 5, o),
                         dtype=torch.uint8, device="cuda")
        adc.adc3_ea_solve(teo, tev, tB, 5, 0.0, 0.0, 1e-7, o, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        roots, reps, st = adc.adc3_ea_solve(teo, tev, tB, 5, 0.0, 0.0, 1e-7, o, workspace=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        inst[tag] = {"time_to_roots_s": dt, "status": st, "iterations": reps[0]["iters"],
                     "iterations_reduced_precision": reps[0]["iters_lowp"] if prec else 0,
                     "max_abs_root_diff_vs_oracle_Eh": vs_oracle(np, roots, g),
                     "max_err_bound_Eh": float(max(r["err_bound"] for r in reps))}
        if ref is None:
            ref = dt
        else:
            inst[tag]["speedup_vs_fp64"] = ref / dt
        print("large workload form: scaled instance %s %.3f s" % (tag, dt), file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    out["scaled_instance"] = inst
    return out


def dfladder_only(adc, torch, reps, precs=(0, 1, 2)):
    """The ladder assembled from the DF factor (adc3_ladder_apply) at the large workload's sigma shape:
    v = 600, X = 1800, 200 rows (5 vectors x 40 occupied), 16 GiB of intermediate, `reps` calls per
    precision after one untimed call; then a 2 GiB device copy for counter calibration."""
    import synth
    v, X, M = 600, 1800, 200
    _, _, B = synth.make_instance(1, v, X, 2, scale=0.05)
    Bvv = torch.as_tensor(B[:, 1:, 1:].copy(), dtype=torch.float64, device="cuda")
    del B
    Z = torch.randn((M, v, v), dtype=torch.float64, device="cuda")
    out = torch.empty_like(Z)
    res = {"mode": "dfladder-only", "nvir": v, "naux": X, "rows": M, "calls_per_precision": reps,
           "flops_per_call": 4.0 * X * M * v ** 3}
    for prec in precs:
        ws = torch.empty(adc.adc3_ladder_workspace_bytes(v, X, M, prec) + (16 << 30), dtype=torch.uint8,
                         device="cuda")
        adc.adc3_ladder_apply(Bvv, Z, precision=prec, out=out, workspace=ws)
        torch.cuda.synchronize()
        adc.adc3_profile_enable(True)
        for _ in range(reps):
            adc.adc3_ladder_apply(Bvv, Z, precision=prec, out=out, workspace=ws)
        torch.cuda.synchronize()
        kind = adc.PROF_LADDER if prec == 0 else adc.PROF_LADDER_LP
        ms, n, fl, by = adc.adc3_profile_query(kind)
        adc.adc3_profile_enable(False)
        peak = (78.6, 157.3, 2500.0)[prec]
        ach = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        res[("fp64", "fp32", "bf16")[prec]] = {"avg_ms": ms / max(n, 1), "achieved_tflops": ach, "peak_tflops": peak,
                                               "frac": ach / peak}
        print("dfladder-only: precision %d done" % prec, file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    x = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    res["copy_bytes_each_way"] = 8 << 28
    return res


def cpu_baseline(shape, nvec):
    """The FP64 oracle's sigma build on the host: nvec ADC(3) sigma vectors on a
    synthetic instance of the truncated-basis shape (one-time intermediates not timed)."""
    import numpy as np

    import synth
    from oracle.adc_cs import Problem
    o, v, X = shape
    eo, ev, B = synth.make_instance(o, v, X, 1)
    P = Problem(eo, ev, B)
    P.m11(3)
    P.coupling_z(3)
    r = np.random.default_rng(0).standard_normal((nvec, P.dim()))
    t0 = time.perf_counter()
    P.sigma(r, 3)
    dt = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    # the oracle's whole solve of the tiny dense workload (o=4, v=20, X=60: every ADC(3) intermediate,
    # the dense 1620 x 1620 matrix and its full diagonalisation)
    p1, eo1, ev1, B1 = synth.preset("tiny-dense")
    t1 = time.perf_counter()
    M = Problem(eo1, ev1, B1).dense(3)
    np.linalg.eigvalsh(0.5 * (M + M.T))
    tiny_s = time.perf_counter() - t1
    return {"value": nvec / dt, "unit": "sigma-builds/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d ADC(3) sigma vectors, o=%d v=%d X=%d (the SS-FNO/NAF basis shape of the workload), "
                      "NumPy FP64; intermediates built once, untimed; %.2f s" % (nvec, o, v, X, dt),
            "compare_with": "sigma_adc3_isolated (the same sigma shape on the GPU)",
            "time_to_roots_tiny_dense_s": tiny_s, "host": host_info()}


def host_info():
    """CPU model, logical CPUs and the BLAS NumPy links (for the CPU baseline record)."""
    import numpy as np
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = ""
    try:
        cfg = np.show_config(mode="dicts")
        b = cfg.get("Build Dependencies", {}).get("blas", {})
        blas = "%s %s" % (b.get("name", ""), b.get("version", ""))
    except Exception:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas.strip(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2511_05897_amd as adc
    import synth

    d = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")  # noqa: E731
    if a.sigma_only:
        # ADC(3) sigma builds in the SS-FNO/NAF basis shape of the default workload
        e2, v2, B2 = synth.make_instance(20, 200, 128, 1)
        ctx = adc.Context(d(e2), d(v2), d(B2), 3, nroots=0, precision=a.sigma_precision)
        r = torch.randn((5, ctx.N), dtype=torch.float64, device="cuda")
        out = torch.empty_like(r)
        for _ in range(a.sigma_reps):
            ctx.sigma(r, out, precision=a.sigma_precision)
        torch.cuda.synchronize()
        # plain copy of known size: 2 GiB read + 2 GiB written
        x = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "sigma-only", "sigma_calls": a.sigma_reps, "nvec": 5, "precision": a.sigma_precision,
                          "ladder_flops_per_launch": 2.0 * 100 * 200 ** 4, "copy_bytes_each_way": 8 << 28}))
        return
    if a.dfladder_only:
        print(json.dumps(dfladder_only(adc, torch, a.sigma_reps,
                                       tuple(int(x) for x in a.dfladder_precs.split(",") if x.strip()))))
        return
    p, eo, ev, B = synth.preset(a.workload, scale=a.scale)
    teo, tev, tB = d(eo), d(ev), d(B)
    del B
    nroots = p["nroots"]
    opts = adc.adc3_default_opts()
    ws = torch.empty(adc.adc3_ea_solve_workspace_bytes(p["nocc"], p["nvir"], p["naux"], nroots, opts),
                     dtype=torch.uint8, device="cuda")
    run = lambda: adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"],  # noqa: E731
                                    opts, workspace=ws)
    # the ladder tuner settles its shapes in a first, untimed solve with the bases one after another, so that
    # its trial launches are timed without the other bases' kernels running beside them
    ot = adc.adc3_default_opts()
    ot.lockstep = 0
    adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], ot, workspace=ws)
    print("tuner settled (one basis at a time, untimed)", file=sys.stderr, flush=True)
    for w in range(a.warmup):
        roots, reps, st = run()
        print("warmup %d done: roots %s status %d" % (w, np.array2string(roots, precision=8), st),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    adc.adc3_profile_enable(True)
    nsig = 0
    nsig3 = 0
    t0 = time.perf_counter()
    for k in range(a.steps):
        roots, reps, st = run()
        nsig += sum(r["sigma_builds"] for r in reps)
        nsig3 += sum(r["sigma_builds_final"] for r in reps)
        print("step %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lad_ms, lad_n, lad_f, lad_b = adc.adc3_profile_query(adc.PROF_LADDER)
    lad_bound = adc.adc3_profile_query_bound(adc.PROF_LADDER)
    sig_ms, sig_n, _, _ = adc.adc3_profile_query(adc.PROF_SIGMA)
    setup_ms, setup_n, _, _ = adc.adc3_profile_query(adc.PROF_SETUP)
    dav_ms, _, _, _ = adc.adc3_profile_query(adc.PROF_DAVIDSON)
    eig_ms, eig_n, _, _ = adc.adc3_profile_query(adc.PROF_EIG)
    adc.adc3_profile_enable(False)
    vk, xk = reps[0]["nvir_kept"], reps[0]["naux_kept"]
    gold = oracle_golden(golden_name(a.workload, a.scale))

    # isolated ADC(3) sigma builds (blocks of nroots vectors) in a basis of the truncated shape
    iso = None
    if a.sigma_reps > 0:
        try:
            e2, v2, B2 = synth.make_instance(p["nocc"], vk, xk, 1, scale=a.scale)
            ctx = adc.Context(d(e2), d(v2), d(B2), 3, nroots=0)
            r = torch.randn((nroots, ctx.N), dtype=torch.float64, device="cuda")
            out = torch.empty_like(r)
            ctx.sigma(r, out)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for _ in range(a.sigma_reps):
                ctx.sigma(r, out)
            torch.cuda.synchronize()
            sdt = time.perf_counter() - s0
            iso = {"value": a.sigma_reps * nroots / sdt, "unit": "sigma-builds/s", "nvec_per_call": nroots,
                   "shape": {"nocc": p["nocc"], "nvir": vk, "naux": xk}}
            print("isolated ADC(3) sigma: %.0f sigma-builds/s" % iso["value"], file=sys.stderr, flush=True)
            ctx.close()
            del ctx
        except Exception as e:  # reported, never silent
            iso = {"error": str(e)}

    # the same solve with reduced-precision sigma (FP64 residual correction), vs the FP64 roots
    mixed = {}
    if not a.no_mixed:
        for prec, tag, peak in ((1, "fp32", 157.3), (2, "bf16", 2500.0)):
            try:
                om = adc.adc3_default_opts()
                om.precision = prec
                wsm = torch.empty(adc.adc3_ea_solve_workspace_bytes(p["nocc"], p["nvir"], p["naux"], nroots, om),
                                  dtype=torch.uint8, device="cuda")
                # one untimed solve first, as for the FP64 steps: the ladder tuner times its candidates
                # on the first call of each shape, with the bases one after another
                om.lockstep = 0
                adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], om, workspace=wsm)
                om.lockstep = -1
                torch.cuda.synchronize()
                adc.adc3_profile_enable(True)
                m0 = time.perf_counter()
                rm, repm, stm = adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"],
                                                  om, workspace=wsm)
                torch.cuda.synchronize()
                mdt = time.perf_counter() - m0
                lms, ln, lf, lb = adc.adc3_profile_query(adc.PROF_LADDER_LP)
                lbound = adc.adc3_profile_query_bound(adc.PROF_LADDER_LP)
                adc.adc3_profile_enable(False)
                del wsm
                ach = lf / (lms * 1e-3) / 1e12 if lms > 0 else 0.0
                mixed[tag] = {"time_to_roots_s": mdt, "speedup_vs_fp64": (dt / a.steps) / mdt, "status": stm,
                              "max_abs_root_diff_vs_fp64_Eh": float(np.abs(rm - roots).max()),
                              "max_abs_root_diff_vs_oracle_Eh": vs_oracle(np, rm, gold),
                              "max_err_bound_Eh": float(max(r["err_bound"] for r in repm)),
                              "root_diff_vs_fp64_Eh": [float(x) for x in (rm - roots)],
                              "lowp_phase_root_error_Eh": [float(r["omega_lowp"] - r["omega_uncorr"]) for r in repm],
                              "ladder": {"launches": ln, "avg_launch_ms": lms / max(ln, 1),
                                         "achieved_tflops": ach, "peak_tflops": peak, "frac": ach / peak,
                                         "bound_time_frac": lbound / lms if lms > 0 else None}}
                print("mixed precision %s: %.3f s to the roots" % (tag, mdt), file=sys.stderr, flush=True)
            except Exception as e:
                mixed[tag] = {"error": str(e)}
        try:
            mixed["ladder_dominated_davidson"] = mixed_ladder_dominated(adc, d, torch, np)
            print("mixed precision: ladder-dominated Davidson done", file=sys.stderr, flush=True)
        except Exception as e:
            mixed["ladder_dominated_davidson"] = {"error": str(e)}

    # the timed steps run the library's default engine: the five roots' truncated bases solved together,
    # each on a host thread and stream of its own (their ADC(2) solves, then their ADC(3) solves); here the
    # same solve with one basis at a time, and with the lockstep block Davidson, for comparison
    lockstep = None
    if not a.no_lockstep:
        try:
            ol = adc.adc3_default_opts()
            ol.lockstep = 0
            wsl = torch.empty(adc.adc3_ea_solve_workspace_bytes(p["nocc"], p["nvir"], p["naux"], nroots, ol),
                              dtype=torch.uint8, device="cuda")
            adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], ol, workspace=wsl)
            torch.cuda.synchronize()
            adc.adc3_profile_enable(True)
            l0 = time.perf_counter()
            rl, repl, stl = adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], ol,
                                              workspace=wsl)
            torch.cuda.synchronize()
            ldt = time.perf_counter() - l0
            iso_ms, iso_n, iso_f, _ = adc.adc3_profile_query(adc.PROF_LADDER)
            iso_bound = adc.adc3_profile_query_bound(adc.PROF_LADDER)
            one_phases = {"setup": adc.adc3_profile_query(adc.PROF_SETUP)[0],
                          "davidson": adc.adc3_profile_query(adc.PROF_DAVIDSON)[0],
                          "sigma": adc.adc3_profile_query(adc.PROF_SIGMA)[0], "ladder": iso_ms,
                          "large_eig": adc.adc3_profile_query(adc.PROF_EIG)[0]}
            adc.adc3_profile_enable(False)
            iso_ach = iso_f / (iso_ms * 1e-3) / 1e12 if iso_ms > 0 else 0.0
            lockstep = {"time_to_roots_s": ldt, "default_speedup_vs_this": ldt / (dt / a.steps), "status": stl,
                        "sigma_builds": sum(r["sigma_builds"] for r in repl),
                        "max_abs_root_diff_vs_default_Eh": float(np.abs(rl - roots).max()),
                        "workspace_GB": wsl.numel() / 1e9,
                        "default_workspace_GB": ws.numel() / 1e9 if ws is not None else None,
                        "phases_ms": one_phases,
                        # the sigma ladder's launches in this solve run one at a time: the kernel's own rate
                        "ladder_roofline": {"achieved": iso_ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                            "frac": iso_ach / PEAK_FP64_TFLOPS, "launches": iso_n,
                                            "avg_launch_ms": iso_ms / max(iso_n, 1),
                                            "flops_per_launch": iso_f / max(iso_n, 1),
                                            "bound_time_frac": iso_bound / iso_ms if iso_ms > 0 else None}}
            print("one basis at a time: %.3f s to the roots" % ldt, file=sys.stderr, flush=True)
            del wsl
            torch.cuda.empty_cache()
        except Exception as e:
            lockstep = {"error": str(e)}

    lock_engine = None
    if not a.no_lockstep:
        try:
            ok = adc.adc3_default_opts()
            ok.lockstep = 1
            wsk = torch.empty(adc.adc3_ea_solve_workspace_bytes(p["nocc"], p["nvir"], p["naux"], nroots, ok),
                              dtype=torch.uint8, device="cuda")
            adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], ok, workspace=wsk)
            torch.cuda.synchronize()
            k0 = time.perf_counter()
            rk, repk, stk = adc.adc3_ea_solve(teo, tev, tB, nroots, p["fno_thresh"], p["naf_thresh"], p["conv"], ok,
                                              workspace=wsk)
            torch.cuda.synchronize()
            kdt = time.perf_counter() - k0
            lock_engine = {"time_to_roots_s": kdt, "default_speedup_vs_this": kdt / (dt / a.steps), "status": stk,
                           "sigma_builds": sum(r["sigma_builds"] for r in repk),
                           "max_abs_root_diff_vs_default_Eh": float(np.abs(rk - roots).max()),
                           "max_abs_root_diff_vs_oracle_Eh": vs_oracle(np, rk, gold),
                           "workspace_GB": wsk.numel() / 1e9}
            print("lockstep engine: %.3f s to the roots" % kdt, file=sys.stderr, flush=True)
            del wsk
            torch.cuda.empty_cache()
        except Exception as e:
            lock_engine = {"error": str(e)}

    # the same workload with B scaled into the weakly correlated regime (SS-FNO then truncates)
    variant = None
    if a.variant_scale > 0:
        try:
            pv, eov, evv, Bv = synth.preset(a.workload, scale=a.variant_scale)
            tBv = d(Bv)
            adc.adc3_ea_solve(d(eov), d(evv), tBv, nroots, pv["fno_thresh"], pv["naf_thresh"], pv["conv"],
                              opts, workspace=ws)
            torch.cuda.synchronize()
            v0 = time.perf_counter()
            rv, repv, stv = adc.adc3_ea_solve(d(eov), d(evv), tBv, nroots, pv["fno_thresh"], pv["naf_thresh"],
                                              pv["conv"], opts, workspace=ws)
            torch.cuda.synchronize()
            vdt = time.perf_counter() - v0
            variant = {"scale": a.variant_scale, "time_to_roots_s": vdt,
                       "max_abs_root_diff_vs_oracle_Eh": vs_oracle(np, rv, oracle_golden(golden_name(a.workload,
                                                                                                    a.variant_scale))),
                       "sigma_builds_per_s": sum(r["sigma_builds"] for r in repv) / vdt,
                       "roots": [float(x) for x in rv], "status": stv,
                       "nvir_kept": [r["nvir_kept"] for r in repv], "naux_kept": [r["naux_kept"] for r in repv]}
            print("weak-correlation variant: %.3f s to the roots" % vdt, file=sys.stderr, flush=True)
            del tBv
        except Exception as e:
            variant = {"error": str(e)}

    achieved = lad_f / (lad_ms * 1e-3) / 1e12 if lad_ms > 0 else 0.0
    # The sigma ladder's rate: its launches in the comparison solve, which runs one basis at a time, so that
    # a launch's HIP-event interval is its own run.  In the timed steps the five bases run concurrently on
    # streams of their own, and an interval also holds the time the launch waits behind the other bases'
    # kernels (the kernel trace of the timed steps shows kernel-only durations equal to the ones here);
    # those figures are kept under timed_steps_events.
    lr = (lockstep or {}).get("ladder_roofline")
    rf = ({"achieved": lr["achieved"], "launches": lr["launches"], "avg_launch_ms": lr["avg_launch_ms"],
           "flops_per_launch": lr["flops_per_launch"], "bound_time_frac": lr["bound_time_frac"],
           "measured_in": "the one-basis-at-a-time solve after the timed steps (same kernels and shapes)"}
          if lr else
          {"achieved": achieved, "launches": lad_n, "avg_launch_ms": lad_ms / max(lad_n, 1),
           "flops_per_launch": lad_f / max(lad_n, 1), "bound_time_frac": lad_bound / lad_ms if lad_ms > 0 else None,
           "measured_in": "the timed steps"})
    src_hash, traffic = ladder_traffic()
    learned = None
    if not a.no_learned:
        try:
            learned = learned_study(adc, d, torch, np)
        except Exception as e:
            learned = {"error": str(e)}
    learned_full = None
    if a.learned_full:
        del ws
        ws = None
        torch.cuda.empty_cache()
        try:
            learned_full = learned_full_size(adc, d, torch, np, 0.3)
        except Exception as e:
            learned_full = {"error": str(e)}
    batched = None
    if a.batched > 0:
        ws = None
        torch.cuda.empty_cache()
        try:
            batched = batched_study(adc, d, torch, np, a.batched,
                                    ((1, "lockstep"),) if a.batched_lockstep_only else
                                    ((0, "threads_cold_tuner"), (1, "lockstep"), (0, "threads")))
        except Exception as e:
            batched = {"error": str(e)}
    large_form = None
    if not a.no_large_form:
        ws = None
        torch.cuda.empty_cache()
        try:
            large_form = large_workload_form(adc, d, torch, np)
        except Exception as e:
            large_form = {"error": str(e)}
    large = None
    if a.large_mixed > 0:
        ws = None
        torch.cuda.empty_cache()
        try:
            precs = tuple(int(x) for x in a.large_mixed_precs.split(",") if x.strip())
            ref = [float(x) for x in a.large_mixed_ref.split(",") if x.strip()] or None
            large = large_mixed_study(adc, d, torch, np, a.large_mixed, precs, ref)
        except Exception as e:
            large = {"error": str(e)}
    line = {
        "metric": "sigma-builds/s (whole SS-FNO-EA-ADC(3) solve) + time-to-5-roots, FP64, 1 GPU",
        "value": nsig / dt,
        "unit": "sigma-builds/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "time_to_roots_s": dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded DF factor and orbital energies)",
        "config": {"workload": a.workload, "nocc": p["nocc"], "nvir": p["nvir"], "naux": p["naux"],
                   "seed": p["seed"], "nroots": nroots, "fno_thresh": p["fno_thresh"],
                   "naf_thresh": p["naf_thresh"], "conv": p["conv"], "scale": a.scale,
                   "nvir_kept": [r["nvir_kept"] for r in reps], "naux_kept": [r["naux_kept"] for r in reps]},
        "roots": [float(x) for x in roots],
        "status": st,
        # against the FP64 oracle's stored roots of the same workload (tests/golden); the bound is the sum
        # of the final FP64 residual norms of the eigenvalues in each root (eq 30's three terms)
        "max_abs_root_diff_vs_oracle_Eh": vs_oracle(np, roots, gold),
        "oracle_golden_conv": gold["oracle_conv"] if gold else None,
        "max_err_bound_Eh": float(max(r["err_bound"] for r in reps)),
        # the sigma builds above mix the cheap ADC(2) solves (canonical and truncated) with the ADC(3) ones;
        # these count the ADC(3) sigma vectors alone over the same timed wall time
        "sigma_builds_per_step": nsig / a.steps,
        "sigma_builds_adc3_per_step": nsig3 / a.steps,
        "sigma_adc3_per_s_whole_solve": nsig3 / dt,
        "roofline": {"kernel": "sigma ladder (ladder_f64t_kernel; ladder_f64_kernel for row tiles of <= 32 rows)",
                     "bound": "mfma",
                     "achieved": rf["achieved"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": rf["achieved"] / PEAK_FP64_TFLOPS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_detail": traffic, "kernel_source_hash": src_hash,
                     "bound_time_frac": rf["bound_time_frac"],
                     "launches": rf["launches"], "avg_launch_ms": rf["avg_launch_ms"],
                     "flops_per_launch": rf["flops_per_launch"], "measured_in": rf["measured_in"],
                     # the same time against F_lad,min = min(4 X o v^3 n_v, executed) per block (the stored pair
                     # blocks execute about o v^4 n_v flops, below the assembled form's when 4 X > v)
                     "frac_vs_min_factorisation": (rf["achieved"] / PEAK_FP64_TFLOPS) * min_factor(xk, vk, p["nocc"]),
                     "timed_steps_events": {"achieved": achieved, "frac": achieved / PEAK_FP64_TFLOPS,
                                            "launches": lad_n, "avg_launch_ms": lad_ms / max(lad_n, 1),
                                            "flops_per_launch": lad_f / max(lad_n, 1),
                                            "bound_time_frac": lad_bound / lad_ms if lad_ms > 0 else None}},
        # phase times from HIP events: in the timed steps the bases' phases run concurrently and their
        # intervals (each including the wait behind the other bases' kernels) add up past the wall time, so
        # the per-phase split is taken from the one-basis-at-a-time solve, and the timed steps' sums are
        # kept beside it
        "phases_ms_per_step": dict((lockstep or {}).get("phases_ms") or {},
                                   measured_in="the one-basis-at-a-time solve (phases one after another)"),
        "phases_ms_per_step_summed_over_streams": {"setup": setup_ms / a.steps, "davidson": dav_ms / a.steps,
                                                   "sigma": sig_ms / a.steps, "ladder": lad_ms / a.steps,
                                                   "large_eig": eig_ms / a.steps},
        "sigma_adc3_isolated": iso,
        "davidson_engine": "the five per-root bases each on a host thread and stream of its own (library default)",
        "one_basis_at_a_time": lockstep,
        "lockstep_engine": lock_engine,
        "mixed_precision": mixed,
        "variant_weak_correlation": variant,
        "learned_preconditioner": learned,
    }
    if learned_full is not None:
        line["learned_full_size"] = learned_full
    if batched is not None:
        line["batched"] = batched
    if large_form is not None:
        line["large_workload_form"] = large_form
    if large is not None:
        line["large_mixed_precision"] = large
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline((p["nocc"], vk, xk), nroots)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
