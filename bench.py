"""Benchmark of the space-time Galerkin TDBIE hot path on one MI355X.

Workload: the 5120-triangle icosphere with 64 graded temporal bases on [0, 8] (every input seeded
and synthetic, resident in device memory before the timed region).

One step = the FP64 assembly of every block A_{k,i} of the block-Hessenberg system (geometry,
time-kernel tables, band layout, regular and singular triangle pairs) and the plane-pulse
right-hand side.  The headline value is assembly quadrature evaluations per second over the
timed steps (one evaluation = one (x_q, y_q', k, i) with |x_q - y_q'| inside supp psi_{k,i},
counted over unordered triangle pairs).

After the timed steps, each once and within a wall-clock budget: the CPU oracle on a bounded
sample of the same workload, the block matvec, the FGMRES solve to a relative residual of 1e-8
with the recursive block-Hessenberg preconditioner (Algorithm 1), the mixed-precision form
(FP64 quadrature, FP32 storage and FP32 inner products, FP64 solver) with its error against FP64, the
field off the surface, the learned preconditioner (trained on the GPU, then used in FGMRES) with
the batched right-hand sides, the uneven-mesh group assembly (one regular-pair launch over eight
spheres), the same sphere on an equidistant grid with and without the copies of equal blocks, and
the deterministic mode.  One JSON line is printed at the end (or on SIGTERM, with what has been
measured by then).  `--config5` runs instead the learned preconditioner's training on pairs from
ten random spheres and tori and the solve of the 20480-triangle torus.

`--copy-calibration` runs only a plain 1 GiB device copy (the reference kernel that scales the
FETCH_SIZE / WRITE_SIZE hardware counters into HBM bytes).
"""
import argparse
import hashlib
import json
import os
import signal
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6          # MI355X, published
HBM_PEAK_GBS = 8000.0
# Algorithmic FP64 flops of one quadrature evaluation (FMA = 2): the two Chebyshev series of
# psi and tilde psi with their shared recurrence, 4 (D + 1), and the weight and the
# accumulation into the local sums, 12 -- about 80 at degree D = 16.  The kernel runs at D = 14
# (4 * 15 + 12 = 72); the figure 80 is kept as the per-evaluation work of the method.
FLOPS_PER_QUAD_EVAL = 80
REGULAR_KERNEL = "k_regular_tile"
KERNEL_SOURCE = os.path.join(ROOT, "paper_1503_07221_amd", "csrc", "k_assemble.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere5120_graded64")
    ap.add_argument("--budget-s", type=float, default=330.0,
                    help="wall-clock seconds after which no further optional leg starts")
    ap.add_argument("--precond", default="2,10", help="Algorithm 1 inner iterations per level ('' = none)")
    ap.add_argument("--restart", type=int, default=300)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-it", type=int, default=300)
    ap.add_argument("--skip-solve", action="store_true", help="no solve legs (profiling)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="approximate CPU seconds of the oracle sample (split over regular and singular pairs)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner leg")
    ap.add_argument("--lp-steps", type=int, default=300,
                    help="Adam steps (batch 8, lr 1e-3) of the learned preconditioner, then half as many at 5e-4")
    ap.add_argument("--lp-layers", type=int, default=4, help="message-passing layers of the learned preconditioner")
    ap.add_argument("--lp-restart", type=int, default=600, help="FGMRES restart of the learned solve")
    ap.add_argument("--lp-max-it", type=int, default=2000, help="iteration limit of the learned solve")
    ap.add_argument("--no-potential", action="store_true", help="skip the field evaluation leg")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-meshes group assembly leg")
    ap.add_argument("--no-deterministic", action="store_true", help="skip the deterministic-mode leg")
    ap.add_argument("--no-equal-blocks", action="store_true",
                    help="skip the equidistant-grid leg (equal blocks copied against integrated)")
    ap.add_argument("--batch-rhs", type=int, default=32,
                    help="right-hand sides of the batched learned solve (0 = skip the batched leg)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--config5", action="store_true",
                    help="only the learned-preconditioner experiment on the 20480-triangle torus (about 12 min)")
    ap.add_argument("--c5-geometries", type=int, default=10, help="random spheres and tori of the training pairs")
    ap.add_argument("--c5-pairs", type=int, default=2000, help="residual/correction pairs over all geometries")
    ap.add_argument("--c5-epochs", type=float, default=3.0, help="passes over the pairs (batch 8)")
    ap.add_argument("--c5-layers", type=int, default=4, help="message-passing layers of the network")
    ap.add_argument("--c5-restart", type=int, default=600, help="FGMRES restart of the learned torus solve")
    ap.add_argument("--c5-learned-it", type=int, default=2400, help="iteration limit of the learned torus solve")
    ap.add_argument("--c5-alg1-it", type=int, default=120, help="iteration limit of the Algorithm 1 torus solve")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 27                                   # 2^27 doubles = 1 GiB
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                      "dispatches": 3}))


def source_digest():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def counted_traffic(workload, launches_quad):
    """HBM bytes per launch of the regular kernel from the committed counter summary, when it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{REGULAR_KERNEL}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_source_sha256_16") != source_digest():
            return None
        fetch = float(vals["fetch_kib_per_dispatch"]) * 1024 * float(vals["fetch_scale"])
        write = float(vals["write_kib_per_dispatch"]) * 1024 * float(vals["write_scale"])
        return fetch + write
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, seconds, quad_regular, quad_singular):
    """The oracle in fast mode (plain C + OpenMP over triangle pairs, FP64, -O3, the same
    quadrature rules, its own uniform-grid tabulation of the time kernels) on seeded samples of
    the workload's unordered triangle pairs: regular pairs and singular (coincident, edge, vertex)
    pairs are timed separately, each for about half of `seconds`; the time of the whole assembly
    is the table build plus each kind's time per quad-eval times its exact count."""
    import numpy as np
    import oracle
    xyz, tri = cfg["mesh"]
    E = len(tri)
    rng = np.random.default_rng(7)
    sets = [set(t) for t in tri]
    vt = {}
    for e, t in enumerate(tri):
        for v in t:
            vt.setdefault(int(v), []).append(e)
    singular = sorted({(min(a, b), max(a, b)) for lst in vt.values() for a in lst for b in lst})
    order = rng.permutation(len(singular))
    singular = [singular[s] for s in order]
    t0 = time.perf_counter()
    tables = oracle.fast_tables(xyz, cfg["grid"], cfg["cutoff"])
    t_tables = time.perf_counter() - t0

    def regular_pairs(n):
        taus, sigs = [], []
        while len(taus) < n:
            a, b = (int(x) for x in rng.integers(0, E, 2))
            if a < b and not (sets[a] & sets[b]):
                taus.append(a); sigs.append(b)
        return np.array(taus), np.array(sigs)

    def sample(kind, n):
        if kind == "regular":
            return regular_pairs(n)
        sel = singular[:min(n, len(singular))]
        return np.array([s[0] for s in sel]), np.array([s[1] for s in sel])

    def timed(taus, sigs):
        t0 = time.perf_counter()
        q, _ = oracle.local_batch(xyz, tri, taus, sigs, cfg["grid"], kind=cfg["cutoff"], tables=tables)
        return q, time.perf_counter() - t0

    res = {}
    for kind in ("regular", "singular"):
        n = 64
        taus, sigs = sample(kind, n)
        q, dt = timed(taus, sigs)
        while dt < 0.05 * seconds and not (kind == "singular" and n >= len(singular)):
            n *= 4
            taus, sigs = sample(kind, n)
            q, dt = timed(taus, sigs)
        if dt < 0.25 * seconds and not (kind == "singular" and n >= len(singular)):
            n = int(n * 0.5 * seconds / max(dt, 1e-3))
            taus, sigs = sample(kind, n)
            q, dt = timed(taus, sigs)
        res[kind] = (len(taus), q, dt)
    (nr, qr, tr), (ns, qs, ts) = res["regular"], res["singular"]
    est = t_tables + quad_regular * tr / qr + quad_singular * ts / qs
    return {"value": (quad_regular + quad_singular) / est, "unit": "quad-evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"oracle fast mode: kernel tables {t_tables:.1f} s, {nr} random regular pairs ({qr} "
                       f"quad-evals, {tr:.1f} s) and {ns} random singular pairs ({qs} quad-evals, {ts:.1f} s) of "
                       f"{cfg['name']}; the whole FP64 assembly ({quad_regular + quad_singular} quad-evals) "
                       f"extrapolated from them: {est:.0f} s"),
            "extrapolated_assembly_s": est}


def sample_entries(ctx, cfg, n, seed):
    """Seeded (k, i, j, l) inside the Hessenberg band (i in k-5 .. k+1) for entry comparisons."""
    import numpy as np
    rng = np.random.default_rng(seed)
    M, N = len(cfg["mesh"][0]), len(cfg["grid"])
    k = rng.integers(0, N, n)
    i = np.clip(k - rng.integers(-1, 6, n), 0, N - 1)
    j = rng.integers(0, M, n)
    l = rng.integers(0, M, n)
    return k, i, j, l


def uneven_leg(tb):
    """Eight geodesic spheres (frequency 4..16: 320 to 5120 triangles) with 16 to 64 graded bases,
    assembled one after the other and then as one group (one context and stream each, the regular
    pairs of all eight in one launch)."""
    import numpy as np
    from workloads import geodesic_sphere, graded_grid
    nus = [4, 5, 6, 7, 8, 10, 12, 16]
    ctxs = []
    for r, nu in enumerate(nus):
        c = tb.Context(0, own_stream=True)
        c.set_mesh(*geodesic_sphere(nu))
        c.set_time_grid(graded_grid(16 + (64 - 16) * r // 7, 8.0, seed=30 + r))
        ctxs.append(c)
    for c in ctxs:                                            # warm-up (and tile-shape timing)
        c.assemble()
    tb.assemble_group(ctxs)
    t0 = time.perf_counter()
    quad = 0
    for c in ctxs:
        quad += c.assemble()["quad_evals"]
    seq = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    reps = tb.assemble_group(ctxs)
    grp = (time.perf_counter() - t0) * 1e3
    assert sum(r["quad_evals"] for r in reps) == quad
    for c in ctxs:
        c.close()
    print(f"# uneven meshes: 8 assemblies {seq:.0f} ms one after the other, {grp:.0f} ms as one group",
          file=sys.stderr, flush=True)
    return {"meshes": [20 * nu * nu for nu in nus], "time_bases": [16 + (64 - 16) * r // 7 for r in range(8)],
            "quad_evals": int(quad), "sequential_ms": seq, "group_ms": grp,
            "sequential_quad_evals_per_s": quad / (seq * 1e-3), "group_quad_evals_per_s": quad / (grp * 1e-3)}


def equal_blocks_leg(tb, cfg):
    """The workload's mesh with 64 equidistant bases on the same [0, T]: FP64 assembly integrating
    every block against the assembly that copies the equal blocks of the inner nodes (eq.
    (relationAtildeBlock)); time, quadrature points integrated, and the largest difference of
    200000 sampled entries relative to the largest sampled entry."""
    import numpy as np
    from workloads import equidistant_grid
    xyz, tri = cfg["mesh"]
    grid = equidistant_grid(len(cfg["grid"]), float(cfg["grid"][-1]))
    c = tb.Context(0)
    c.set_mesh(xyz, tri)
    c.set_time_grid(grid, "bump")
    sample = sample_entries(c, {"mesh": cfg["mesh"], "grid": grid}, 200000, 7)
    res = {}
    for reuse in (0, 1):
        c.set_block_reuse(reuse)
        r = [c.assemble(tb.FP64) for _ in range(2)][-1]
        res[reuse] = (r, c.get_entries(*sample))
        print(f"# equal blocks {'copied' if reuse else 'integrated'}: assembly {r['ms_total']:.1f} ms "
              f"(regular {r['ms_regular']:.1f}, copies {r['ms_reuse']:.1f})", file=sys.stderr, flush=True)
    c.close()
    (r0, e0), (r1, e1) = res[0], res[1]
    return {"workload": f"{cfg['name'].split('_')[0]}_eq{len(grid)}", "time_bases": len(grid),
            "integrated": {"ms": r0["ms_total"], "ms_regular": r0["ms_regular"], "quad_evals": int(r0["quad_evals"])},
            "copied": {"ms": r1["ms_total"], "ms_regular": r1["ms_regular"], "ms_copies": r1["ms_reuse"],
                       "quad_evals": int(r1["quad_evals"]), "blocks_copied": int(r1["blocks_reused"])},
            "speedup": r0["ms_total"] / r1["ms_total"],
            "sampled_max_rel_diff": float(np.abs(e1 - e0).max() / max(np.abs(e0).max(), 1e-300))}


def deterministic_leg(tb, cfg, ref_entries, sample):
    """The deterministic mode on the workload: two FP64 assemblies (each a scale pass and a
    fixed-point pass), their time, whether the sampled entries are bitwise equal, and their largest
    difference from the ordinary assembly relative to the largest sampled entry."""
    import numpy as np
    c = tb.Context(0, deterministic=True)
    c.set_mesh(*cfg["mesh"])
    c.set_time_grid(cfg["grid"], cfg["cutoff"])
    reps, ents = [], []
    for _ in range(2):
        reps.append(c.assemble(tb.FP64))
        ents.append(c.get_entries(*sample))
    c.close()
    print(f"# deterministic: assembly {reps[-1]['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    return {"ms": reps[-1]["ms_total"], "quad_evals": int(reps[-1]["quad_evals"]),
            "bitwise_equal_runs": bool(np.array_equal(ents[0].view(np.int64), ents[1].view(np.int64))),
            "max_rel_diff_vs_ordinary": float(np.abs(ents[1] - ref_entries).max() / np.abs(ref_entries).max())}


def potential_leg(ctx, tb, alpha, cfg):
    """The scattered field of the FP64 solution on a 257 x 257 grid of the plane z = 0 over
    [-3, 3]^2 (66049 points, as in the paper's field evaluation) at 40 equally spaced times."""
    import numpy as np
    import torch
    T = float(cfg["grid"][-1])
    g1 = np.linspace(-3.0, 3.0, 257)
    X, Y = np.meshgrid(g1, g1, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    times = np.linspace(T / 40, T, 40)
    u = ctx.potential_dl(alpha, pts[:1024], times[:8])       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = ctx.potential_dl(alpha, pts, times)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    E = len(cfg["mesh"][1])
    evals = len(pts) * len(times) * E * 7
    print(f"# potential: {len(pts)} points x {len(times)} times in {ms:.0f} ms", file=sys.stderr, flush=True)
    return {"points": int(len(pts)), "times": int(len(times)), "ms": ms,
            "point_time_per_s": len(pts) * len(times) / (ms * 1e-3),
            "quadrature_evals_per_s": evals / (ms * 1e-3), "max_abs_u": float(u.abs().max())}


def mixed_leg(ctx, tb, cfg, args, g, alpha64, inner, n, time_matvec, rep64, solve64):
    """The mixed form on the same inputs.  Assembly: FP64 quadrature and FP32 storage, its speed and
    its entry and matvec error against the FP64 assembly.  Solve: the outer FGMRES iteration and its true residual on the FP64 operator,
    Algorithm 1's inner products on an FP32 copy of the FP64 band, to the same 1e-8 on the FP64
    system."""
    import numpy as np
    import torch
    xr = torch.randn(n, dtype=torch.float64, device="cuda:0",
                     generator=torch.Generator(device="cuda:0").manual_seed(11))
    ctx.assemble(tb.FP64)
    y64 = ctx.matvec(xr).clone()
    ks, is_, js, ls = sample_entries(ctx, cfg, 200000, 5)
    e64 = ctx.get_entries(ks, is_, js, ls)
    mreps = [ctx.assemble(tb.MIXED) for _ in range(2)]
    mrep = mreps[-1]
    print(f"# mixed: assembly {mrep['ms_total']:.1f} ms (regular {mrep['ms_regular']:.1f})", file=sys.stderr,
          flush=True)
    y32 = ctx.matvec(xr)
    e32 = ctx.get_entries(ks, is_, js, ls)
    mv32 = time_matvec()
    res = {"assembly_ms": mrep["ms_total"], "regular_ms": mrep["ms_regular"],
           "value": mrep["quad_evals"] / (mrep["ms_total"] * 1e-3), "matrix_bytes": int(mrep["bytes_matrix"]),
           "fp64_assembly_ms": rep64["ms_total"], "matvec_ms": mv32,
           "matvec_GBps": mrep["bytes_matrix"] / (mv32 * 1e-3) / 1e9,
           "matvec_rel_err_vs_fp64": float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64)),
           "entry_max_err_rel_to_max_entry": float(np.max(np.abs(e32 - e64)) / np.max(np.abs(e64)))}
    ctx.assemble(tb.FP64)
    if alpha64 is not None and not args.skip_solve and inner:
        a32, srep = ctx.solve(g, tol=args.tol, restart=args.restart, max_it=args.max_it, precond_inner=inner,
                              inner_fp32=True)
        r = g - ctx.matvec(a32)
        r64 = float(torch.linalg.norm(r) / torch.linalg.norm(g))
        res["solve"] = {"kind": "FP64 outer iteration and residual, FP32 inner products of Algorithm 1",
                        "ms": srep["ms"], "iterations": int(srep["iterations"]),
                        "rel_residual_fp64_operator": r64, "converged": bool(srep["converged"]),
                        "solution_rel_diff_vs_fp64": float(torch.linalg.norm(a32 - alpha64) / torch.linalg.norm(alpha64))}
        if solve64:
            res["solve"]["speedup_vs_fp64_solve"] = solve64["ms"] / srep["ms"]
        print(f"# mixed solve: {srep['ms']:.0f} ms ({srep['iterations']} it), residual {r64:.2e} on the FP64 "
              f"operator", file=sys.stderr, flush=True)
    return res


def learned_leg(ctx, tb, args, g, alpha_ref, solve_ref, budget):
    """Train the learned preconditioner on the FP64 operator, then solve with it (kernels launched
    one by one, then as a captured graph per iteration); solutions are compared with the Algorithm 1
    solution alpha_ref."""
    import numpy as np
    import torch
    ctx.assemble(tb.FP64)
    ctx.lp_init(args.lp_layers, seed=3)
    hist, trep = ctx.lp_train(steps=args.lp_steps, batch=8, lr=1e-3, seed=4)
    hist2, trep2 = ctx.lp_train(steps=max(1, args.lp_steps // 2), batch=8, lr=5e-4, seed=5)
    hist = np.concatenate([hist, hist2])
    trep = {"ms": trep["ms"] + trep2["ms"], "samples": trep["samples"] + trep2["samples"]}
    print(f"# learned: trained {trep['samples']} residuals in {trep['ms']:.0f} ms, loss {hist[0]:.3f} -> "
          f"{hist[-10:].mean():.3f}", file=sys.stderr, flush=True)
    x = torch.randn_like(g)
    ctx.lp_apply(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        ctx.lp_apply(x)
    e1.record()
    e1.synchronize()
    res = {"layers": args.lp_layers, "hidden": 64, "params": ctx.lp_num_params(), "train_steps": len(hist), "batch": 8,
           "train_ms": trep["ms"], "train_samples": int(trep["samples"]), "loss_first": float(hist[0]),
           "loss_last10": float(hist[-10:].mean()), "apply_ms": e0.elapsed_time(e1) / 10}
    nrm = torch.linalg.norm(alpha_ref)
    for tag in ("fp64",):
        a, srep = ctx.solve(g, tol=args.tol, restart=args.lp_restart, max_it=args.lp_max_it,
                            precond_kind=tb.PRECOND_LEARNED)
        print(f"# learned {tag}: solve {srep['ms']:.1f} ms ({srep['iterations']} it, residual "
              f"{srep['rel_residual']:.2e})", file=sys.stderr, flush=True)
        res[tag] = {"solve_ms": srep["ms"], "iterations": int(srep["iterations"]),
                    "rel_residual": float(srep["rel_residual"]), "converged": bool(srep["converged"]),
                    "solution_rel_diff_vs_alg1_fp64": float(torch.linalg.norm(a - alpha_ref) / nrm)}
        if solve_ref:
            res[tag]["speedup_vs_alg1_fp64_solve"] = solve_ref["ms"] / srep["ms"]
    ctx.assemble(tb.FP64)
    a, srep = ctx.solve(g, tol=args.tol, restart=args.lp_restart, max_it=args.lp_max_it,
                        precond_kind=tb.PRECOND_LEARNED, use_graph=True)
    print(f"# learned fp64, captured iteration: solve {srep['ms']:.1f} ms ({srep['iterations']} it)",
          file=sys.stderr, flush=True)
    res["fp64_graph"] = {"solve_ms": srep["ms"], "iterations": int(srep["iterations"]),
                         "rel_residual": float(srep["rel_residual"]), "converged": bool(srep["converged"]),
                         "solution_rel_diff_vs_alg1_fp64": float(torch.linalg.norm(a - alpha_ref) / nrm)}
    if args.batch_rhs > 0 and budget.allows("batched", 75):
        res["batched"] = batched_leg(ctx, tb, args, res["fp64"]["solve_ms"])
    ctx.assemble(tb.FP64)
    return res


def batched_leg(ctx, tb, args, single_ms):
    """32 plane pulses (seeded directions on S^2, widths uniform in [0.1, 0.3], t0 = 1 + 6 w) on the
    same sphere solved together with the learned preconditioner: one multi-right-hand-side product
    per iteration.  Also the product alone: time per right-hand side for 1 and for 32 vectors."""
    import numpy as np
    import torch
    from workloads.configs import pulse_direction
    ctx.assemble(tb.FP64)
    R = args.batch_rhs
    rng = np.random.default_rng(7)
    G = torch.stack([ctx.rhs_plane_pulse(pulse_direction(1000 + r), 1.0 + 6 * w, w)
                     for r, w in enumerate(rng.uniform(0.1, 0.3, R))])
    X = torch.randn_like(G)
    ctx.matvec_multi(X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        ctx.matvec_multi(X)
    e1.record()
    e1.synchronize()
    multi_ms = e0.elapsed_time(e1) / 3
    A, reps, ok = ctx.solve_multi(G, tol=args.tol, restart=args.lp_restart + 200, max_it=args.lp_max_it,
                                  precond_kind=tb.PRECOND_LEARNED)
    ms = reps[0]["ms"]
    its = [r["iterations"] for r in reps]
    print(f"# batched: {R} right-hand sides in {ms:.0f} ms (iterations {min(its)}..{max(its)}), product "
          f"{multi_ms:.1f} ms for {R} vectors", file=sys.stderr, flush=True)
    return {"rhs": R, "solve_ms": ms, "ms_per_rhs": ms / R, "converged": bool(ok),
            "iterations_min": int(min(its)), "iterations_max": int(max(its)),
            "max_rel_residual": float(max(r["rel_residual"] for r in reps)),
            "speedup_vs_single_learned_solves": single_ms * R / ms,
            "product_ms": multi_ms, "product_ms_per_rhs": multi_ms / R}


class Budget:
    """Wall-clock budget of the optional legs: a leg starts only if its estimated duration fits in
    what is left, so the whole run stays inside the time the caller allows."""

    def __init__(self, seconds):
        self.t0 = time.perf_counter()
        self.seconds = seconds
        self.skipped = []

    def left(self):
        return self.seconds - (time.perf_counter() - self.t0)

    def allows(self, name, estimate_s):
        if self.left() >= estimate_s:
            return True
        self.skipped.append(name)
        print(f"# {name}: skipped ({estimate_s:.0f} s estimated, {self.left():.0f} s of the budget left)",
              file=sys.stderr, flush=True)
        return False


def mean_edge(xyz, tri):
    import numpy as np
    e = np.concatenate([xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 1]],
                        xyz[tri[:, 0]] - xyz[tri[:, 2]]])
    return float(np.linalg.norm(e, axis=1).mean())


def config5(args):
    """The learned preconditioner of the torus workload, trained as that workload states: a
    4-layer network on residual/correction pairs that the method generates on randomly sized
    spheres and tori (residual A e of an error e drawn by the library, correction e), then used
    as FGMRES's variable preconditioner on the 20480-triangle torus with 128 graded bases (mixed
    storage), against Algorithm 1 (2, 10) on the same operator; iterations, time and residual,
    and the residual of the learned solution under the FP64 matrix-free product."""
    import numpy as np
    import torch
    import paper_1503_07221_amd as tb
    from workloads import get_config, graded_grid, icosphere, torus

    t_all = time.perf_counter()
    rng = np.random.default_rng(5)
    per = args.c5_pairs // args.c5_geometries
    geoms, desc = [], []
    t0 = time.perf_counter()
    for gi in range(args.c5_geometries):
        if gi % 2 == 0:
            lev = int(rng.choice([2, 3]))
            rad = float(rng.uniform(0.7, 1.3))
            xyz, tri = icosphere(lev)
            xyz = xyz * rad
            name = f"sphere L{lev} radius {rad:.3f}"
        else:
            R = float(rng.uniform(0.8, 1.2))
            r = R * float(rng.uniform(0.25, 0.45))
            nu = int(rng.choice([24, 32, 40]))
            nv = max(8, int(round(nu * 1.25 * r / R)))
            xyz, tri = torus(nu, nv, R, r)
            name = f"torus {nu}x{nv} R {R:.3f} r {r:.3f}"
        N = int(rng.integers(16, 33))
        T = float(rng.uniform(1.5, 3.0)) * mean_edge(xyz, tri) * (N - 1)
        grid = graded_grid(N, T, seed=100 + gi)
        c = tb.Context(0)
        c.set_mesh(xyz, tri)
        c.set_time_grid(grid, "bump")
        c.assemble(tb.FP64)
        V, Z = c.lp_make_pairs(per, seed=200 + gi)
        geoms.append((c, V, Z))
        desc.append({"mesh": name, "triangles": int(len(tri)), "time_bases": N, "T": T, "pairs": per})
        print(f"# config5: {name}, {len(tri)} triangles, {N} bases on [0, {T:.2f}], {per} pairs",
              file=sys.stderr, flush=True)
    pairs_s = time.perf_counter() - t0
    net = tb.Context(0)
    net.lp_init(args.c5_layers, seed=6)
    steps_total = int(args.c5_epochs * args.c5_pairs / 8)
    chunk = 5
    rounds = max(1, steps_total // (chunk * len(geoms)))
    hist = []
    t0 = time.perf_counter()
    for rd in range(rounds):
        lr = 1e-3 if rd < (2 * rounds) // 3 else 5e-4
        for gi, (c, V, Z) in enumerate(geoms):
            h, _ = net.lp_train_pairs(c, V, Z, steps=chunk, batch=8, lr=lr, seed=1000 * rd + gi)
            hist.append(h)
        if rd % 5 == 0 or rd == rounds - 1:
            print(f"# config5: training round {rd + 1}/{rounds}, loss {np.concatenate(hist[-len(geoms):]).mean():.3f}",
                  file=sys.stderr, flush=True)
    train_s = time.perf_counter() - t0
    hist = np.concatenate(hist)
    params = net.lp_get_params()
    for c, V, Z in geoms:
        c.close()
    del geoms
    net.close()
    torch.cuda.empty_cache()

    cfg = get_config("torus20480_graded128")
    xyz, tri = cfg["mesh"]
    ctx = tb.Context(0)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(cfg["grid"], cfg["cutoff"])
    t0 = time.perf_counter()
    arep = ctx.assemble(tb.MIXED)
    asm_s = time.perf_counter() - t0
    print(f"# config5: torus assembled (mixed) in {asm_s:.1f} s, {arep['quad_evals']:.3e} quad-evals",
          file=sys.stderr, flush=True)
    g = ctx.rhs_plane_pulse(cfg["direction"], cfg["t0"], cfg["width"])
    gn = torch.linalg.norm(g).item()
    ctx.lp_init(args.c5_layers, seed=0)
    ctx.lp_set_params(params)
    out = {"workload": "torus20480_graded128", "precision": "mixed (FP32 storage, FP64 solver)",
           "layers": args.c5_layers,
           "training": {"geometries": desc, "pairs": per * len(desc), "pair_generation_s": pairs_s,
                        "adam_steps": int(len(hist)), "batch": 8, "train_s": train_s,
                        "loss_first": float(hist[:10].mean()), "loss_last": float(hist[-50:].mean())},
           "assembly_s": asm_s, "quad_evals": int(arep["quad_evals"])}

    def progress(tag, every):
        def cb(it, est):
            if it % every == 0:
                print(f"# config5 {tag}: iteration {it}, estimate {est:.3e}", file=sys.stderr, flush=True)
        return cb

    a_l, r_l = ctx.solve(g, tol=1e-8, restart=args.c5_restart, max_it=args.c5_learned_it,
                         precond_kind=tb.PRECOND_LEARNED, progress=progress("learned", 300))
    res_l = torch.linalg.norm(g - ctx.matvec(a_l)).item() / gn
    out["learned"] = {"solver": f"FGMRES({args.c5_restart}) + network", "iterations": int(r_l["iterations"]),
                      "ms": r_l["ms"], "rel_residual": res_l, "converged": bool(r_l["converged"])}
    print(f"# config5 learned: {r_l['iterations']} it, {r_l['ms'] / 1e3:.1f} s, residual {res_l:.3e}",
          file=sys.stderr, flush=True)
    yf, _ = ctx.matvec_free(a_l)
    out["learned"]["rel_residual_fp64_matrix_free"] = torch.linalg.norm(g - yf).item() / gn
    print(f"# config5 learned: FP64 matrix-free residual {out['learned']['rel_residual_fp64_matrix_free']:.3e}",
          file=sys.stderr, flush=True)
    if args.c5_alg1_it > 0:
        a_a, r_a = ctx.solve(g, tol=1e-8, restart=300, max_it=args.c5_alg1_it, precond_inner=(2, 10),
                             progress=progress("alg1", 20))
        res_a = torch.linalg.norm(g - ctx.matvec(a_a)).item() / gn
        out["alg1"] = {"solver": "FGMRES(300) + Algorithm 1 (2, 10)", "iterations": int(r_a["iterations"]),
                       "ms": r_a["ms"], "rel_residual": res_a, "converged": bool(r_a["converged"])}
        print(f"# config5 alg1: {r_a['iterations']} it, {r_a['ms'] / 1e3:.1f} s, residual {res_a:.3e}",
              file=sys.stderr, flush=True)
    out["wall_s"] = time.perf_counter() - t_all
    print(json.dumps({"config5": out}), flush=True)
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.config5:
        config5(args)
        return
    budget = Budget(args.budget_s)
    import numpy as np
    import torch
    import paper_1503_07221_amd as tb
    from workloads import get_config

    cfg = get_config(args.workload)
    xyz, tri = cfg["mesh"]
    grid = cfg["grid"]
    inner = tuple(int(v) for v in args.precond.split(",") if v)
    ctx = tb.Context(0)
    ctx.set_mesh(xyz, tri)
    ctx.set_time_grid(grid, cfg["cutoff"])
    n = len(grid) * len(xyz)
    g = torch.empty(n, dtype=torch.float64, device="cuda:0")
    alpha = torch.empty_like(g)
    out = {}

    def emit(signum=None, frame=None):
        """Print the JSON line with what has been measured so far (also on SIGTERM)."""
        if out.get("_printed"):
            return
        out["_printed"] = True
        line = {k: v for k, v in out.items() if k != "_printed"}
        if budget.skipped:
            line["legs_skipped"] = budget.skipped
        print(json.dumps(line), flush=True)
        if signum is not None:
            sys.exit(124)

    def step():
        """One step: the FP64 assembly of every block and the right-hand side."""
        rep = ctx.assemble(tb.FP64)
        ctx.rhs_plane_pulse(cfg["direction"], cfg["t0"], cfg["width"], out=g)
        return rep

    def time_matvec(launches=20):
        """Average time of a full block matvec y = A x (HIP events on the library's stream)."""
        x = torch.randn(n, dtype=torch.float64, device="cuda:0",
                        generator=torch.Generator(device="cuda:0").manual_seed(12))
        y = torch.empty_like(x)
        for _ in range(3):
            ctx.matvec(x, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            ctx.matvec(x, out=y)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / launches

    def note(tag, rep, srep=None):
        s = f"# {tag}: assembly {rep['ms_total']:.1f} ms (regular {rep['ms_regular']:.1f})"
        if srep:
            s += f", solve {srep['ms']:.1f} ms ({srep['iterations']} it, residual {srep['rel_residual']:.2e})"
        print(s, file=sys.stderr, flush=True)

    # ---- the timed steps: FP64 assembly (the headline) -------------------------------------
    for w in range(args.warmup):
        note(f"warmup {w}", step())
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        rep = step()
        reps.append(rep)
        note(f"step {s}", rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    quad = reps[-1]["quad_evals"]
    quad_reg = reps[-1]["quad_evals_regular"]
    asm_ms = float(np.mean([r["ms_total"] for r in reps]))
    reg_ms = float(np.mean([r["ms_regular"] for r in reps]))
    achieved_tflops = quad_reg * FLOPS_PER_QUAD_EVAL / (reg_ms * 1e-3) / 1e12
    out.update({
        "metric": "assembly quad-evals/s + FGMRES solve time to 1e-8 resid (FP64 vs mixed)",
        "value": quad * args.steps / wall,
        "unit": "quad-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "triangles": int(len(tri)), "vertices": int(len(xyz)),
                   "time_bases": int(len(grid)), "T": float(grid[-1]), "precision": "fp64",
                   "step": "FP64 assembly of every block (tables, layout, regular and singular pairs) "
                           "+ right-hand side"},
        "assembly_ms_events": asm_ms,
        "quad_evals": int(quad),
        "quad_evals_regular": int(quad_reg),
        "assembly_breakdown_ms": {k: float(np.mean([r[k] for r in reps]))
                                  for k in ("ms_tables", "ms_layout", "ms_regular", "ms_singular")},
        "matrix_bytes": int(reps[-1]["bytes_matrix"]),
        "regular_tiles": {"shape": "%dx%d" % ctx.assemble_tuning()[0],
                          "timed_ms_per_launch": {"4x8": ctx.assemble_tuning()[1][0], "8x8": ctx.assemble_tuning()[1][1]}},
        "roofline": {"bound": "alu", "kernel": REGULAR_KERNEL, "achieved": achieved_tflops,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": counted_traffic(cfg["name"], quad_reg),
                     "flops_per_quad_eval": FLOPS_PER_QUAD_EVAL, "launch_ms": reg_ms,
                     "quad_evals_per_launch": int(quad_reg)},
    })
    signal.signal(signal.SIGTERM, emit)

    # ---- the CPU oracle on a bounded sample of the same workload ----------------------------
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds, quad_reg, quad - quad_reg)
        print(f"# cpu baseline: {out['cpu_baseline']['value']:.3e} quad-evals/s "
              f"({out['cpu_baseline']['cores']} threads)", file=sys.stderr, flush=True)

    # ---- the block matvec ------------------------------------------------------------------
    mv_ms = time_matvec()
    out["matvec"] = {"fp64_ms": mv_ms, "fp64_GBps": reps[-1]["bytes_matrix"] / (mv_ms * 1e-3) / 1e9,
                     "hbm_peak_GBps": HBM_PEAK_GBS,
                     "fp64_frac": reps[-1]["bytes_matrix"] / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # ---- the solve to 1e-8 (FP64, Algorithm 1) ----------------------------------------------
    srep = None
    if not args.skip_solve and budget.allows("solve", 40):
        _, srep = ctx.solve(g, tol=args.tol, restart=args.restart, max_it=args.max_it, precond_inner=inner,
                            out=alpha)
        out["solve"] = {"solver": f"FGMRES({args.restart}) + Algorithm 1 {inner}" if inner
                        else f"FGMRES({args.restart})",
                        "ms": srep["ms"], "iterations": int(srep["iterations"]), "matvecs": int(srep["matvecs"]),
                        "rel_residual": float(srep["rel_residual"]), "converged": bool(srep["converged"])}
        print(f"# solve: {srep['ms']:.0f} ms ({srep['iterations']} it, residual {srep['rel_residual']:.2e})",
              file=sys.stderr, flush=True)

    # ---- the mixed form on the same inputs -----------------------------------------------------
    if not args.no_mixed and budget.allows("mixed", 45):
        out["mixed"] = mixed_leg(ctx, tb, cfg, args, g, alpha if srep else None, inner, n, time_matvec,
                                 reps[-1], out.get("solve"))
    if srep and not args.no_potential and budget.allows("potential", 15):
        out["potential"] = potential_leg(ctx, tb, alpha, cfg)
    if not args.no_learned and srep and budget.allows("learned", 110):
        out["learned"] = learned_leg(ctx, tb, args, g, alpha, out.get("solve"), budget)
    if not args.no_uneven and budget.allows("uneven", 30):
        out["uneven"] = uneven_leg(tb)
    if not args.no_equal_blocks and budget.allows("equal_blocks", 25):
        out["equal_blocks"] = equal_blocks_leg(tb, cfg)
    if not args.no_deterministic and budget.allows("deterministic", 20):
        ctx.assemble(tb.FP64)
        sample = sample_entries(ctx, cfg, 200000, 9)
        out["deterministic"] = deterministic_leg(tb, cfg, ctx.get_entries(*sample), sample)
    ctx.close()
    emit()


if __name__ == "__main__":
    main()
