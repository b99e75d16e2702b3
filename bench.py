"""Benchmark: exponential-midpoint steps per second on one MI355X.

Workload (default): the 4,096-atom diamond-like lattice with 13 functions per
atom (53,248 x 53,248 complex K), cut-offs R_HS 10, R_K 16 and R_P 16 bohr,
H = H0 + 0.5 diag(Mulliken charges) rebuilt every step, dt 0.05 a.u.  Every
step rebuilds A = P(X H) (as P(X H0), kept from the set-up, plus X's block
columns scaled by the on-site term: the model's H differs from H0 only on the
diagonal), the 6-term Taylor propagator and K <- U K U^dagger.  The same run
with the full X H product at every step is reported beside it.
Inputs are synthetic and seeded; all of them are resident in HBM before the
timed region starts.

Prints ONE JSON line with steps/s, the roofline of the dominant product
kernel (algorithmic flops per launch over its average HIP-event duration) and
the oracle's CPU rate on a bounded sample.  Beside the FP64 run, on the same
workload: the reduced-precision forms (late Taylor terms in FP32, split BF16
or split FP16) with the learned inverse start, their dipole error against the
FP64 run; the captured-graph step; a batch leg (all 64 clusters of the
batching workload with x/y/z kicks, stepped together by captured graphs, FP64
and FP32, against one system at a time); the 64-atom cluster with multi-step
graphs against eager steps; and FP64 steps/s of the b = 4 lattices (65,536
atoms, and 32,768 atoms at R_K 12) with their kernels' roofline fractions.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
# Identifies the product kernel build whose HBM traffic profiles/traffic.json holds;
# change it whenever the kernel changes so that a stale figure is not reported.
KERNEL_TAG = "q4j-b13-nj2seg-xcdchunk128-tile256-v1"


# The same for the real b = 4 run kernel on the 32,768-atom lattice at R_K 12.
KERNEL_TAG_B4 = "b4j-runs16-pipelined-real-v1"


def measured_traffic(dom, name="traffic.json", tag=KERNEL_TAG, workload=None):
    path = os.path.join(ROOT, "profiles", name)
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if t.get("kernel_tag") != tag or t.get("product") != dom:
        return None
    if workload is not None and t.get("workload") != workload:
        return None
    return t["bytes_per_launch"]
METRIC = "propagation steps/s + block-SpGEMM GFLOP/s (% roofline) at stated dipole error vs FP64"


def per_product_ms(stats):
    """Mean milliseconds per launch of each product kind that ran."""
    return {k: v[1] / v[0] for k, v in stats.items() if v[0]}


def full_xh(s, args, base):
    """The same FP64 run with A = P_P(X H) formed by the full product at every
    step (what a Hamiltonian that changes everywhere costs), against the
    default A0 + X D form."""
    f = gpu_run(s, args, xh_every_step=1)
    n = min(len(base["trace"]), len(f["trace"]))
    induced = np.abs(base["trace"][:n, 1:4] - base["p0"]).max()
    return {"steps_per_s": args.steps / f["elapsed"], "a0_form_speedup": f["elapsed"] / base["elapsed"],
            "dipole_difference_rel": float(np.abs(f["trace"][:n, 1:4] - base["trace"][:n, 1:4]).max() / induced),
            "per_product_ms": per_product_ms(f["stats"])}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(args):
    from paper_1404_5776_amd import synth
    cells = tuple(int(x) for x in args.cells.split("x"))
    s = synth.config2(cells=cells, n_steps=args.steps)
    return s


def gpu_run(s, args, precision="fp64", taylor_low_from=3, use_graph=0, inv_start="block_jacobi",
            mlp_weights=None, xh_every_step=0):
    import torch  # device memory and streams come from torch's runtime
    from paper_1404_5776_amd import rtdm

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = rtdm.Context(0, h_model=s.h_model, h_gain=s.h_gain, precision=precision,
                       taylor_low_from=taylor_low_from, use_graph=use_graph, inv_start=inv_start,
                       xh_every_step=xh_every_step)
    t = time.time()
    ctx.load_system(s, stream)
    log(f"[{precision}] set-up (neighbour lists, schedules, upload) {time.time() - t:.1f} s")
    if mlp_weights is not None:
        rtdm.rtdm_mlp_set_weights(ctx.h, mlp_weights)
    torch.cuda.synchronize()
    t = time.perf_counter()
    iters, res = rtdm.rtdm_build_inverse(ctx.h, stream)
    inv_s = time.perf_counter() - t
    log(f"[{precision}] inverse ({inv_start} start): {iters} iterations, residual {res:.2e}, {inv_s:.2f} s")
    rtdm.rtdm_apply_kick(ctx.h, s.kappa, stream)
    p0 = rtdm.rtdm_observables(ctx.h, stream)[:3]
    sched = {k: rtdm.rtdm_schedule_stats(ctx.h, k) for k in ("XH", "AT", "UK", "WU")}
    if args.warmup:
        rtdm.rtdm_step(ctx.h, s.dt, args.warmup, stream)
    torch.cuda.synchronize()
    rtdm.rtdm_timing(ctx.h, not use_graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = getattr(args, "progress_every", 0)
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done) if chunk > 0 else args.steps - done
        rtdm.rtdm_step(ctx.h, s.dt, n, stream)
        done += n
        if chunk > 0:
            torch.cuda.synchronize()          # long runs report each finished chunk of steps
            log(f"[{precision}] {done}/{args.steps} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {k: rtdm.rtdm_timing_stats(ctx.h, k) for k in ("XH", "AT", "UK", "WU")}
    rtdm.rtdm_timing(ctx.h, False)
    trace = rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    return dict(elapsed=t1 - t0, stats=stats, sched=sched, trace=trace, p0=p0, inv_iters=iters, inv_s=inv_s)


def measured_peaks():
    """Achievable rates on this GPU for context: FP64 GEMM through torch's BLAS
    (8192^3, best of 5) and a device copy of 2 GiB (read + write, best of 5)."""
    import torch
    n = 8192
    a = torch.rand(n, n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, n, dtype=torch.float64, device="cuda")
    torch.matmul(a, b)
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    gemm = 2.0 * n ** 3 / best / 1e12
    del a, b
    x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = 1e30
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    bw = 2.0 * x.numel() * 8 / best / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"fp64_gemm_tflops": gemm, "copy_gb_per_s": bw,
            "note": "torch.matmul float64 8192^3 and a 2 GiB device copy, best of 5; context for the "
                    "published peaks the roofline uses"}


def train_learned_start(b, seeds=(101, 102, 103), cells=(3, 3, 3)):
    """Train the inverse-start network on converged inverses of small lattices
    of the workload's recipe (held-out seeds); returns its weights."""
    from paper_1404_5776_amd import rtdm, synth
    ctx = None
    t = time.time()
    for k, seed in enumerate(seeds):
        sysk = synth.diamond_lattice(cells, b, 10.0, 16.0, seed=seed, k0="local", h_model="mulliken")
        if ctx is None:
            ctx = rtdm.Context(0, inv_tol=1e-12)
            ctx.load_system(sysk)
            rtdm.rtdm_mlp_init(ctx.h, 7)
        else:
            ctx.load_system(sysk)
        rtdm.rtdm_build_inverse(ctx.h)
        rtdm.rtdm_mlp_collect(ctx.h, 4000, 100 + k)
    loss = rtdm.rtdm_mlp_train(ctx.h, 60, 256, 2e-3, 11)
    w = rtdm.rtdm_mlp_get_weights(ctx.h)
    ctx.close()
    log(f"learned start: trained on {len(seeds)} lattices of {cells} cells, loss {loss:.2e}, "
        f"{time.time() - t:.1f} s")
    return w, loss


def batch_leg(args):
    """The 64-cluster workload (log-uniform 50-2,000 atoms, b 4 or 13, R_HS 8,
    R_K 12 bohr, fixed H), every cluster with x, y and z kicks: 192
    propagations.  Batched: one kick-set context per b (each cluster once, as
    a group of a block-diagonal geometry; three K per context sharing one
    propagator), both advanced by one rtdm batch whose captured graph moves
    all propagations graph_steps steps per launch.  Per system: each cluster
    alone in a context of its own with the x kick and captured graphs of the
    same length; its y and z propagations run the same kernels on the same
    patterns, so they are counted at the x kick's time.  FP64 (b = 13 launch
    shapes autotuned on both sides) and FP32."""
    import torch
    from paper_1404_5776_amd import rtdm, synth

    t = time.time()
    clusters = synth.config4_all(n_clusters=args.batch_clusters)
    log(f"batch: {len(clusters)} clusters, {sum(c.n_atoms for c in clusters)} atoms, "
        f"generated in {time.time() - t:.1f} s")
    kicks = [(0.01, 0.0, 0.0), (0.0, 0.01, 0.0), (0.0, 0.0, 0.01)]
    G, n_steps, dt = args.batch_graph_steps, args.batch_steps, clusters[0].dt
    by_b = {b: [c for c in clusters if c.b == b] for b in (4, 13)}
    n_prop = len(kicks) * len(clusters)
    out = {"workload": f"{len(clusters)} random clusters (log-uniform 50-2000 atoms, b 4 or 13, R_HS 8, "
                       f"R_K 12 bohr, fixed H), x/y/z kicks each: {n_prop} propagations; batched as one "
                       f"kick-set context per b stepped by one captured graph per {G} steps",
           "propagations": n_prop, "atoms": int(sum(c.n_atoms for c in clusters)),
           "clusters_by_b": {str(b): len(v) for b, v in by_b.items()}, "steps": n_steps, "graph_steps": G}
    stream = torch.cuda.current_stream()
    for prec in ("fp64", "fp32"):
        tune = prec == "fp64"
        ctxs, shapes = [], {}
        for b, members in by_b.items():
            if not members:
                continue
            ctx = rtdm.Context(0, precision=prec, n_kicks=len(kicks), use_graph=1, graph_steps=G)
            ctx.load_kick_sets(members, kicks, stream)
            rtdm.rtdm_build_inverse(ctx.h, stream)
            rtdm.rtdm_apply_kicks(ctx.h, ctx.kick_vectors, stream)
            ctxs.append(ctx)
        bt = rtdm.rtdm_batch_create([c.h for c in ctxs], G)
        rtdm.rtdm_batch_step(bt, dt, 1, stream)           # the fixed-H propagators
        if tune:
            for ctx in ctxs:
                if ctx.b == 13:
                    shapes["batched_b13"] = rtdm.rtdm_autotune(ctx.h, stream)
        rtdm.rtdm_batch_step(bt, dt, G, stream)           # capture and one replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rtdm.rtdm_batch_step(bt, dt, n_steps, stream)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        rtdm.rtdm_batch_destroy(bt)
        for ctx in ctxs:
            ctx.close()
        t_sys = 0.0
        for c in clusters:
            ctx = rtdm.Context(0, precision=prec, use_graph=1, graph_steps=G)
            ctx.load_system(c, stream)
            rtdm.rtdm_build_inverse(ctx.h, stream)
            rtdm.rtdm_apply_kick(ctx.h, kicks[0], stream)
            rtdm.rtdm_step(ctx.h, dt, 1, stream)
            if tune and c.b == 13:
                rtdm.rtdm_autotune(ctx.h, stream)
            rtdm.rtdm_step(ctx.h, dt, G, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rtdm.rtdm_step(ctx.h, dt, n_steps, stream)
            torch.cuda.synchronize()
            t_sys += time.perf_counter() - t0
            ctx.close()
        t_sys *= len(kicks)
        out[prec] = {"propagation_steps_per_s": n_prop * n_steps / t_batch,
                     "seconds_per_step_all_propagations": t_batch / n_steps,
                     "per_system_propagation_steps_per_s": n_prop * n_steps / t_sys,
                     "speedup_vs_per_system": t_sys / t_batch}
        if shapes:
            out[prec]["autotuned_wpb_row_tile"] = shapes
        log(f"batch {prec}: {out[prec]}")
    return out


def small_leg(args):
    """The 64-atom cluster (b = 4, R_HS 8, R_K 12, fixed H, 100 steps): eager
    steps against steps replayed from captured graphs of graph_steps steps."""
    import torch
    from paper_1404_5776_amd import rtdm, synth

    s = synth.config1()
    stream = torch.cuda.current_stream()
    out = {"workload": f"cluster {s.n_atoms} atoms x {s.b} functions, R_HS {s.R_HS} R_K {s.R_K} bohr, "
                       f"fixed H, EM + Taylor p=5, dt {s.dt}, {s.n_steps} steps",
           "graph_steps": args.small_graph_steps}
    import gc
    traces = {}
    reps = 5
    out["timing"] = (f"median over {reps} consecutive calls of {s.n_steps} steps each (a call of 100 steps "
                     f"lasts about 5 ms, so one host hiccup would otherwise decide it); Python's collector "
                     f"paused while timing")
    for use_graph in (0, 1):
        ctx = rtdm.Context(0, use_graph=use_graph, graph_steps=args.small_graph_steps)
        ctx.load_system(s, stream)
        rtdm.rtdm_reserve_trace(ctx.h, 1 + args.small_graph_steps + reps * s.n_steps)
        rtdm.rtdm_build_inverse(ctx.h, stream)
        rtdm.rtdm_apply_kick(ctx.h, s.kappa, stream)
        rtdm.rtdm_step(ctx.h, s.dt, 1 + args.small_graph_steps, stream)      # U, capture, one replay
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        try:
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                rtdm.rtdm_step(ctx.h, s.dt, s.n_steps, stream)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
        finally:
            gc.enable()
        traces[use_graph] = rtdm.rtdm_dipole_trace(ctx.h)
        ctx.close()
        out["graph_steps_per_s" if use_graph else "eager_steps_per_s"] = s.n_steps / float(np.median(times))
    out["speedup_graph_vs_eager"] = out["graph_steps_per_s"] / out["eager_steps_per_s"]
    out["bit_identical_trace"] = bool(np.array_equal(traces[0][:, :6], traces[1][:, :6]))
    log(f"small system: {out}")
    return out


def b4_leg(args):
    """FP64 steps/s of the b = 4 lattices, with the roofline fraction of their
    dominant product kernel: the 65,536-atom lattice (R_K 12) and the
    32,768-atom lattice at R_K 12, both with the Mulliken on-site H.  On the
    65,536-atom lattice also the mixed-precision + learned form (late Taylor
    terms in FP32, network-started inverse) against the FP64 run: steps/s
    with and without the inverse build, and its dipole error."""
    from paper_1404_5776_amd import synth

    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup = args.b4_steps, 2
    out = {}
    makers = {"65536": ("lattice65536_rk12", lambda: synth.config5(n_steps=sub.steps)),
              "32768": ("lattice32768_rk12", lambda: synth.config3(12.0, n_steps=sub.steps))}
    for key, make in (makers[k] for k in args.b4_lattices.split(",") if k):
        t = time.time()
        s = make()
        log(f"b4 {key}: generated in {time.time() - t:.1f} s")
        r = gpu_run(s, sub)
        stats = r["stats"]
        dom = max(stats, key=lambda k: stats[k][1])
        n_l, ms, fl = stats[dom]
        ach = fl / n_l / (ms / 1e3 / n_l) / 1e12
        roof = {"bound": "mfma", "kernel": f"k_spgemm_b4j ({dom} product)", "achieved": ach,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "avg_launch_ms": ms / n_l, "flops_per_launch": fl / n_l,
                "traffic": measured_traffic(dom, "traffic_b4.json", KERNEL_TAG_B4, key),
                "traffic_unit": "bytes per launch"}
        if roof["traffic"] is not None:
            roof["beyond_l2_gb_per_s"] = roof["traffic"] / (ms / 1e3 / n_l) / 1e9
            roof["beyond_l2_frac_of_hbm_peak"] = roof["beyond_l2_gb_per_s"] / 8000.0
        step_s = r["elapsed"] / sub.steps
        out[key] = {"atoms": s.n_atoms, "b": s.b, "R_HS": s.R_HS, "R_K": s.R_K, "steps": sub.steps,
                    "steps_per_s": sub.steps / r["elapsed"],
                    "inverse": {"iterations": r["inv_iters"], "seconds": r["inv_s"]},
                    "steps_per_s_with_inverse_build": {f"n{n}": n / (r["inv_s"] + n * step_s) for n in (10, 100)},
                    "per_product_ms": per_product_ms(stats),
                    "roofline": roof}
        log(f"b4 {key}: {out[key]['steps_per_s']:.2f} steps/s, {dom} {out[key]['roofline']['frac']:.3f} of peak")
        if key == "lattice32768_rk12" and not args.no_full_xh:
            out[key]["full_xh_product"] = full_xh(s, sub, r)
            log(f"b4 {key} full X H product: {out[key]['full_xh_product']}")
        if key == "lattice32768_rk12" and not args.no_b4_forms:
            n = len(r["trace"])
            induced = np.abs(r["trace"][:, 1:4] - r["p0"]).max()
            forms = {}
            for form in ("fp32_taylor", "bf16x3_taylor"):
                f = gpu_run(s, sub, precision=form, taylor_low_from=args.low_from)
                forms[form] = {"steps_per_s": sub.steps / f["elapsed"], "speedup_vs_fp64": r["elapsed"] / f["elapsed"],
                               "dipole_error_vs_fp64": float(np.abs(f["trace"][:n, 1:4] - r["trace"][:n, 1:4]).max()
                                                             / induced),
                               "per_product_ms": per_product_ms(f["stats"])}
            out[key]["late_taylor_forms"] = forms
            log(f"b4 {key} late-Taylor forms: {forms}")
        if key == "lattice65536_rk12" and not args.no_learned:
            w, loss = train_learned_start(4)
            m = gpu_run(s, sub, precision="fp32_taylor", taylor_low_from=args.low_from, inv_start="learned",
                        mlp_weights=w)
            n = min(len(r["trace"]), len(m["trace"]))
            induced = np.abs(r["trace"][:n, 1:4] - r["p0"]).max()
            m_step = m["elapsed"] / sub.steps
            out[key]["fp32_taylor_learned"] = {
                "steps_per_s": sub.steps / m["elapsed"], "speedup_vs_fp64": r["elapsed"] / m["elapsed"],
                "dipole_error_vs_fp64": float(np.abs(m["trace"][:n, 1:4] - r["trace"][:n, 1:4]).max() / induced),
                "compared_steps": int(n),
                "inverse": {"iterations": m["inv_iters"], "seconds": m["inv_s"]},
                "steps_per_s_with_inverse_build": {f"n{k}": k / (m["inv_s"] + k * m_step) for k in (10, 100)},
                "speedup_with_inverse_build": {f"n{k}": (r["inv_s"] + k * step_s) / (m["inv_s"] + k * m_step)
                                               for k in (10, 100)},
                "training_loss": loss}
            log(f"b4 {key} fp32_taylor + learned: {out[key]['fp32_taylor_learned']}")
    return out


def cpu_baseline(s, target_s: float):
    """Oracle product rate on a bounded row sample of each product kind, scaled to steps/s."""
    from oracle import oracle as O

    st = O.setup(s)
    rng = np.random.default_rng(0)
    b = s.b
    M = O.BSM(st.pat_p, b, rng.uniform(-1, 1, (st.pat_p.nnzb, b, b)) + 0j)
    Kc = M if st.pat_k is st.pat_p else O.BSM(st.pat_k, b, rng.uniform(-1, 1, (st.pat_k.nnzb, b, b)) + 0j)
    kinds = {"XH": (M, st.H0, st.pat_p, 0), "AT": (M, M, st.pat_p, 0), "UK": (M, Kc, st.pat_k, 0),
             "WU": (Kc, M, st.pat_k, 1)}
    per_kind = target_s / len(kinds)
    rate = {}
    total_rows = 0
    for k, (A, B, pc, ob) in kinds.items():
        rows = 8
        while True:
            lo = s.n_atoms // 2 - rows // 2
            t = time.perf_counter()
            _, trip = O.spgemm(A, B, pc, op_b=ob, rows=(lo, lo + rows))
            dt = time.perf_counter() - t
            if dt > 0.25 * per_kind or rows >= s.n_atoms:
                break
            rows = min(s.n_atoms, rows * 4)
        rate[k] = trip / dt
        total_rows += rows
    return rate, total_rows


def study_precision(args):
    """Reduced-precision forms on the 32,768-atom b = 4 lattice at each K
    cut-off: dipole and Tr(KS) error against the FP64 run on the same GPU,
    and steps/s.  Prints one JSON line."""
    from paper_1404_5776_amd import synth
    forms = [f for f in args.sweep_forms.split(",") if f]
    out = {"study": "precision", "workload": "diamond lattice 32768 atoms x 4 functions, R_HS 10 bohr, "
                                            "Mulliken on-site H, EM + Taylor p=5, dt 0.05",
           "steps": args.steps, "warmup": args.warmup, "taylor_low_from": args.low_from, "cutoffs": []}
    for R_K in (float(x) for x in args.cutoffs.split(",")):
        t = time.time()
        s = synth.config3(R_K, n_steps=args.steps)
        log(f"R_K {R_K}: generated in {time.time() - t:.1f} s")
        base = gpu_run(s, args)
        tr0, p0 = base["trace"], base["p0"]
        n = len(tr0)
        induced = np.abs(tr0[:, 1:4] - p0).max()
        row = {"R_K": R_K, "fp64_steps_per_s": args.steps / base["elapsed"],
               "triples_per_product": {k: v[1] for k, v in base["sched"].items()}, "forms": {}}
        for form in forms:
            r = gpu_run(s, args, precision=form, taylor_low_from=args.low_from)
            tr = r["trace"]
            row["forms"][form] = {
                "steps_per_s": args.steps / r["elapsed"],
                "dipole_error_vs_fp64": float(np.abs(tr[:n, 1:4] - tr0[:n, 1:4]).max() / induced),
                "trks_error_vs_fp64": float(np.abs(tr[:n, 4] - tr0[:n, 4]).max() / abs(tr0[0, 4]))}
            log(f"R_K {R_K} {form}: {row['forms'][form]}")
        out["cutoffs"].append(row)
    print(json.dumps(out))


def study_learned(args):
    """The 65,536-atom b = 4 lattice (R_K 12): iterations and time of the
    inverse build from the block-Jacobi and from the learned start (network
    trained on three held-out 216-atom lattices of the R_K 16 recipe), and
    steps/s with and without the build at 10 and 100 steps.  One JSON line."""
    import torch
    from paper_1404_5776_amd import synth
    torch.cuda.init()                     # torch's runtime first: it provides the streams
    t = time.time()
    s = synth.config5(n_steps=args.steps)
    log(f"{s.name}: generated in {time.time() - t:.1f} s")
    w, loss = train_learned_start(s.b)
    base = gpu_run(s, args)
    lrn = gpu_run(s, args, inv_start="learned", mlp_weights=w)
    step_s = base["elapsed"] / args.steps
    out = {"study": "learned", "workload": "diamond lattice 65536 atoms x 4 functions, R_HS 10, R_K 12 bohr, "
                                          "Mulliken on-site H, EM + Taylor p=5, dt 0.05",
           "training_loss": loss, "steps": args.steps,
           "block_jacobi": {"iterations": base["inv_iters"], "inverse_s": base["inv_s"]},
           "learned": {"iterations": lrn["inv_iters"], "inverse_s": lrn["inv_s"]},
           "steps_per_s": args.steps / base["elapsed"],
           "dipole_trace_identical_within": float(np.abs(lrn["trace"][:, 1:4] - base["trace"][:, 1:4]).max())}
    for n in (10, 100):
        out[f"steps_per_s_with_build_n{n}"] = {
            "block_jacobi": n / (base["inv_s"] + n * step_s), "learned": n / (lrn["inv_s"] + n * step_s)}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", default="8x8x8", help="diamond conventional cells (8 atoms each)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0, help="oracle sample budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32_taylor,bf16x3_taylor,fp16x2_taylor",
                    help="reduced-precision forms run beside FP64 (comma list, empty for none)")
    ap.add_argument("--no-learned", action="store_true", help="forms use the block-Jacobi inverse start")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-full-xh", action="store_true",
                    help="skip the runs with the full X H product at every step (A0 + X D form only)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the GEMM / copy rate measurement")
    ap.add_argument("--no-b4-forms", action="store_true",
                    help="skip the FP32 / BF16x3 late-Taylor runs on the 32,768-atom b = 4 lattice")
    ap.add_argument("--batch-clusters", type=int, default=64,
                    help="clusters of the batch leg, the first of the 64-cluster list (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=32, help="timed steps of the batch leg")
    ap.add_argument("--batch-graph-steps", type=int, default=16, help="steps per captured graph, batch leg")
    ap.add_argument("--small-graph-steps", type=int, default=16,
                    help="steps per captured graph, 64-atom cluster leg (0: skip the leg)")
    ap.add_argument("--b4-steps", type=int, default=10, help="timed steps of the b = 4 lattices (0: skip)")
    ap.add_argument("--b4-lattices", default="65536,32768", help="b = 4 lattices to run (atom counts)")
    ap.add_argument("--leg", choices=["batch", "small", "b4"], default=None,
                    help="run only this leg of the benchmark and print its JSON object (for profiling)")
    ap.add_argument("--low-from", type=int, default=3, help="first Taylor order in reduced precision in the *_taylor forms")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (read + write) before the workload, "
                         "so hardware byte counters can be scaled against a known size")
    ap.add_argument("--study", choices=["precision", "learned"], default=None,
                    help="instead of the benchmark line: the precision sweep on the 32,768-atom lattice, or "
                         "the learned inverse start on the 65,536-atom lattice (one JSON line each)")
    ap.add_argument("--cutoffs", default="8,12,16,20", help="K cut-offs of the precision study (bohr)")
    ap.add_argument("--progress-every", type=int, default=0, metavar="STEPS",
                    help="time the steps in calls of this many, logging after each (0: one call)")
    ap.add_argument("--sweep-forms", default="fp32,fp32_taylor,bf16x3,bf16x3_taylor,fp16x2,fp16x2_taylor",
                    help="forms of the precision study beside FP64 (comma list)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; the multi-GPU path (spatial "
                                   "domain decomposition with halo exchange) is a design, not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.study == "precision":
        study_precision(args)
        return
    if args.study == "learned":
        study_learned(args)
        return

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)        # one elementwise kernel: reads MIB MiB, writes MIB MiB
        torch.cuda.synchronize()
        log(f"copy calibration: 3 elementwise copies of {args.calibrate_copy} MiB")
        del x, y

    if args.leg:
        import torch
        torch.cuda.init()
        print(json.dumps({"leg": args.leg, **{"batch": batch_leg, "small": small_leg, "b4": b4_leg}[args.leg](args)}))
        return

    t = time.time()
    s = make_workload(args)
    log(f"workload {s.name}: {s.n_atoms} atoms, b={s.b}, generated in {time.time() - t:.1f} s")
    base = gpu_run(s, args)
    elapsed, stats, sched, trace, p0 = base["elapsed"], base["stats"], base["sched"], base["trace"], base["p0"]
    steps_per_s = args.steps / elapsed

    def compare(run):
        n = min(len(trace), len(run["trace"]))
        induced = np.abs(trace[:n, 1:4] - p0).max()
        err = np.abs(run["trace"][:n, 1:4] - trace[:n, 1:4]).max()
        return err / induced, err, n

    forms = []
    weights = None
    if args.forms:
        if not args.no_learned:
            weights, loss = train_learned_start(s.b)
        for form in args.forms.split(","):
            r = gpu_run(s, args, precision=form, taylor_low_from=args.low_from,
                        inv_start="learned" if weights is not None else "block_jacobi", mlp_weights=weights)
            e_rel, e_abs, n = compare(r)
            forms.append({"precision": form, "taylor_low_from": args.low_from,
                          "inverse_start": "learned" if weights is not None else "block_jacobi",
                          "steps_per_s": args.steps / r["elapsed"], "speedup_vs_fp64": elapsed / r["elapsed"],
                          "dipole_error_vs_fp64": e_rel, "dipole_error_abs": e_abs, "compared_steps": int(n),
                          "inverse_iterations": r["inv_iters"], "inverse_s": r["inv_s"],
                          "per_product_ms": per_product_ms(r["stats"])})
            log(f"form {form}: {forms[-1]['steps_per_s']:.3f} steps/s, dipole error {e_rel:.2e}")
    graph = None
    if not args.no_graph:
        g = gpu_run(s, args, use_graph=1)
        graph = {"steps_per_s": args.steps / g["elapsed"], "speedup_vs_eager": elapsed / g["elapsed"],
                 "bit_identical_trace": bool(np.array_equal(g["trace"][:, :6], trace[:, :6]))}
        log(f"graph: {graph}")
    fullxh = None
    if not args.no_full_xh:
        fullxh = full_xh(s, args, base)
        log(f"full X H product: {fullxh}")
    learned = None
    if weights is not None:
        learned = {"inverse_iterations_block_jacobi": base["inv_iters"],
                   "inverse_s_block_jacobi": base["inv_s"],
                   "inverse_iterations_learned": forms[0]["inverse_iterations"] if forms else None,
                   "inverse_s_learned": forms[0]["inverse_s"] if forms else None,
                   "training_loss": loss,
                   "training_data": "converged inverses (residual 1e-12) of three 216-atom lattices of the "
                                    "same recipe with held-out seeds"}
    batch = batch_leg(args) if args.batch_clusters > 0 else None
    small = small_leg(args) if args.small_graph_steps > 0 else None
    b4 = b4_leg(args) if args.b4_steps > 0 else None
    peaks = None if args.no_peaks else measured_peaks()
    if peaks:
        log(f"measured peaks: {peaks}")

    # dominant product kernel: the kind with the most kernel time
    dom = max(stats, key=lambda k: stats[k][1])
    n_l, ms, fl = stats[dom]
    avg_s = ms / 1e3 / n_l
    achieved = fl / n_l / avg_s / 1e12
    tot_fl = sum(v[2] for v in stats.values())
    tot_ms = sum(v[1] for v in stats.values())
    flops_per_step = tot_fl / args.steps

    traffic = measured_traffic(dom)
    roofline = {"bound": "mfma", "kernel": f"k_spgemm_q4j<13, NJ=2> ({dom} product)", "achieved": achieved,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "avg_launch_ms": avg_s * 1e3, "flops_per_launch": fl / n_l}
    if traffic is not None:
        # the roof that binds in practice: bytes beyond L2 (hardware counters of this
        # kernel build) per launch over this run's launch time, against the copy rate
        rate = traffic / avg_s / 1e9
        roofline["beyond_l2_gb_per_s"] = rate
        roofline["beyond_l2_frac_of_hbm_peak"] = rate / 8000.0
        if peaks:
            roofline["beyond_l2_frac_of_measured_copy"] = rate / peaks["copy_gb_per_s"]

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t = time.time()
        threads = O.set_threads(0)
        per_step = {"XH": 1, "AT": 4, "UK": 1, "WU": 1}
        b3 = float(s.b) ** 3
        flops_per_trip = {k: 8 * b3 for k in per_step}       # the oracle multiplies complex128 blocks

        def rate_of(seconds):
            rate, rows = cpu_baseline(s, seconds)
            sec = sum(per_step[k] * sched[k][1] / rate[k] for k in per_step)
            gf = sum(per_step[k] * sched[k][1] * flops_per_trip[k] for k in per_step) / sec / 1e9
            return 1.0 / sec, gf, rows

        v_all, gf_all, rows = rate_of(args.cpu_seconds)
        O.set_threads(1)
        v_one, gf_one, rows1 = rate_of(args.cpu_seconds / 8)
        O.set_threads(threads)
        cpu = {"value": v_all, "unit": "steps/s", "cores": threads, "kind": "oracle",
               "sample": f"oracle masked block products (complex128) on {rows} output atom rows of the "
                         f"XH, AT, UK and WU products of this workload, triples/s per kind scaled by the "
                         f"per-step triple counts (1 XH + 4 AT + 1 UK + 1 WU); {time.time() - t:.0f} s wall "
                         f"with the single-thread sample",
               "gflops": gf_all, "single_thread": {"value": v_one, "gflops": gf_one, "rows": rows1},
               "gflops_note": "complex128 flops of the oracle's products (8 b^3 per triple), the GPU's "
                              "real-specialised count is lower"}

    out = {
        "metric": METRIC,
        "value": steps_per_s,
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
        "config": {"workload": f"diamond lattice {s.n_atoms} atoms x {s.b} functions, R_HS {s.R_HS} "
                               f"R_P {s.R_P} R_K {s.R_K} bohr, Mulliken on-site H, EM + Taylor p=5, "
                               f"dt {s.dt}",
                   "atoms": s.n_atoms, "b": s.b},
        "spgemm_gflops": tot_fl / (tot_ms / 1e3) / 1e9,
        "spgemm_tflop_per_step": flops_per_step / 1e12,
        "accuracy": "FP64 path; equals the FP64 oracle within 1e-10 relative in the parity tests, "
                    "so its dipole error vs FP64 is at that level",
        "roofline": roofline,
        "per_product_ms": per_product_ms(stats),
        "trace_last": trace[-1, :6].tolist() if len(trace) else None,
        "cpu_baseline": cpu,
        "precision_forms": forms,
        "graph": graph,
        "full_xh_product": fullxh,
        "learned_start": learned,
        "batch": batch,
        "small_system": small,
        "b4": b4,
        "measured_peaks": peaks,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
