"""Benchmark of the Galerkin BIE Poisson-Boltzmann hot path on one MI355X.

One step = one full pass of the path on the ~500k-panel workload: cluster
tree, near-field assembly (singular cubature, near-singular pairs replaced by
the learned surrogate where its calibrated error passes the stated gate) with
preconditioner factors, right-hand side, mixed-precision flexible GMRES to a
1e-6 true residual of that operator (FP32 FMM/near field inside, FP64
outside), and the solvation energy.  The surrogate is trained once before the
timed steps (time reported separately).  Inputs
(mesh, charges) are host arrays handed to the library, as its C ABI defines.

value = FMM matvec throughput [Mpanels/s] of the mixed-precision operator,
from HIP events around every matvec issued inside the timed steps.  The same
line reports the GMRES time-to-1e-6 of the mixed and the plain FP64 paths,
the dominant kernel against its roofline, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM matvec Mpanels/s + GMRES time-to-1e-6 (mixed+MLP vs FP64) at 500k panels"
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of k_spmv<float4> from rocprofv3 FETCH_SIZE + WRITE_SIZE
# (calibrated with a device copy of known size); None until measured for the
# kernel as it stands
TRAFFIC_SPMV = 1332068352   # FETCH 640,595.2 KiB x 2.0000 + WRITE 19,657.6 KiB x 1.0 per launch
# acceptance parameter of the treecode energy (rho_l / R <= theta) and its
# order cap (terms |b| <= min(p_l, 6))
ENERGY_THETA = 0.5
ENERGY_PMAX = 6
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoid500k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=12)
    ap.add_argument("--mlp-epochs", type=int, default=120,
                    help="training epochs of the near-field surrogate (before the timed steps)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


PARAMS = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8, quad_duffy=7,
              near_ratio=2.0, tol=1e-6, max_iter=200, max_outer=5, inner_tol=5e-7,
              precond=3,   # block-diagonal preconditioner over consecutive leaves, <= 32 panels
              rhs_theta=0.5, rhs_pmax=6)   # right-hand side by the reverse treecode
MLP_GATE = 0.05         # stated per-pair error tolerance of the gated near field


def train_surrogate(F, torch, pairs_per_mesh=1000000, epochs=120):
    """Train the near-field network on cubature-labelled pairs of the
    81,920-panel multi-charge sphere and the ~200k-panel globule."""
    from synth import workload
    Xs, Ts, As = [], [], []
    t0 = time.perf_counter()
    for name in ("kirkwood2", "globule200k"):
        w = workload(name)
        h = F.Handle().build_tree(w["verts"], w["tris"]).assemble_nearfield()
        X, T, A = h.mlp_dataset(pairs_per_mesh)
        Xs.append(X.clone()); Ts.append(T.clone()); As.append(A.clone())
        h.close()
    X, T, A = torch.cat(Xs), torch.cat(Ts), torch.cat(As)
    t1 = time.perf_counter()
    h = F.Handle()
    hist = h.mlp_train(X.contiguous(), T.contiguous(), A.contiguous(), epochs=epochs, batch=4096,
                       lr=3e-3, seed=5)
    t2 = time.perf_counter()
    blob = h.mlp_get_weights()
    # per-pair error on the held-out rows (every tenth) against the cubature:
    # max over the six outputs of |pred - true| / (|full integral| + 0.1 rms)
    val = torch.arange(9, X.shape[0], 10, device=X.device)
    Y = h.mlp_forward(X[val].contiguous()).cpu().numpy()
    t = T[val].cpu().numpy()
    full = A[val, 2:].cpu().numpy()
    cls = A[val, 0].cpu().numpy()
    h.close()
    rms = np.sqrt((full ** 2).mean(0))
    err = (np.abs(Y - t) / (np.abs(full) + 0.1 * rms)).max(1)
    err0 = (np.abs(t) / (np.abs(full) + 0.1 * rms)).max(1)
    edges = [0.0, 0.003, 0.01, 0.03, 0.1, 0.3, 1.0, np.inf]
    hist_err = {}
    for c, name in enumerate(("edge", "vertex", "close")):
        e, e0 = err[cls == c], err0[cls == c]
        hist_err[name] = {"pairs": int(e.size),
                          "p50": float(np.percentile(e, 50)), "p90": float(np.percentile(e, 90)),
                          "p99": float(np.percentile(e, 99)),
                          "p50_without_network": float(np.percentile(e0, 50)),
                          "histogram": {"edges": [float(x) for x in edges[:-1]] + ["inf"],
                                        "counts": np.histogram(e, bins=edges)[0].tolist()}}
    return blob, {"pairs": int(X.shape[0]), "epochs": epochs, "data_s": t1 - t0, "train_s": t2 - t1,
                  "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                  "heldout_error_vs_cubature": hist_err}


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def m2l_flops(h):
    """algorithmic M2L flops per matvec (2 channels, 2 flops per multiply-add)"""
    return 2.0 * h.tree_info().m2l_flops_fp


def cpu_baseline(w, rows):
    """FP64 oracle (dense rows, O(N) per row) on a sample of rows of the
    same mesh; the full dense matvec takes N times one row."""
    from oracle import dense
    from oracle.geometry import panels
    P = panels(w["verts"], w["tris"])
    rng = np.random.default_rng(7)
    x = rng.standard_normal(2 * P.n)
    sel = rng.choice(P.n, rows, replace=False)
    eps = w["eps_out"] / w["eps_in"]
    t0 = time.perf_counter()
    for r in sel:
        dense.rows_matvec(P, eps, w["kappa"], x, np.array([r]))
    dt = (time.perf_counter() - t0) / rows
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        threads = os.cpu_count()
    return {"value": 1e-6 / dt, "unit": "Mpanels/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d rows of the dense FP64 oracle matvec (all %d source panels per "
                      "row, singular rules for touching/close pairs) on the same mesh; "
                      "rate = 1/(time per row), i.e. the full O(N^2) matvec rate; "
                      "numpy single-threaded (%d host threads available)"
                      % (rows, P.n, threads)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU; --gpus %d is not supported "
              "(the path shards by contiguous Morton ranges of leaves; not built here)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2110_13778_amd as F
    from synth import workload

    torch.cuda.set_device(0)
    w = workload(args.workload)
    N = len(w["tris"])
    dev = "cuda:0"
    stream = torch.cuda.current_stream()

    log("workload %s: %d panels, %d charges" % (args.workload, N, len(w["q"])))
    blob, mlp_info = train_surrogate(F, torch, epochs=args.mlp_epochs)
    log("surrogate trained on %d pairs in %.1f s" % (mlp_info["pairs"], mlp_info["train_s"]))

    def run(prec, profile, direct=False):
        mlp = dict(mlp_mode=F.MLP_GATED, mlp_gate_tol=MLP_GATE) if prec == F.MIXED else {}
        prm = dict(PARAMS, rhs_theta=0.0) if direct else PARAMS
        h = F.Handle(precision=prec, eps_in=w["eps_in"], eps_out=w["eps_out"],
                     kappa=w["kappa"], **prm, **mlp)
        if prec == F.MIXED:
            h.mlp_set_weights(blob)
        h.set_profiling(profile)
        t0 = time.perf_counter()
        h.build_tree(w["verts"], w["tris"])
        t1 = time.perf_counter()
        h.assemble_nearfield()
        t2 = time.perf_counter()
        x = torch.zeros(2 * N, dtype=torch.float64, device=dev)
        code, info = h.solve(w["xq"], w["q"], x)
        t3 = time.perf_counter()
        if direct:
            E = h.solvation_energy(x, w["xq"], w["q"])
        else:
            E = h.solvation_energy_treecode(x, w["xq"], w["q"], ENERGY_THETA, p_max=ENERGY_PMAX)
        t4 = time.perf_counter()
        gated = h.mlp_stats() if prec == F.MIXED else (0, 0)
        pr = h.profile()
        setup = {k: pr[k] for k in ("ms_tree", "ms_classify", "ms_surrogate", "ms_singular", "ms_fmm_setup",
                                    "ms_precond")}
        return h, x, dict(code=code, mlp_gated=gated[0], mlp_candidates=gated[1], setup_stages_ms=setup,
                          t_rhs_ms=info.t_rhs_ms, t_iterations_ms=info.t_solve_ms, tree_ms=1e3 * (t1 - t0), assemble_ms=1e3 * (t2 - t1),
                          solve_ms=1e3 * (t3 - t2), energy_ms=1e3 * (t4 - t3),
                          total_ms=1e3 * (t4 - t0), iters=info.inner_iterations,
                          outer=info.outer_iterations, mv64=info.matvecs_fp64,
                          mv32=info.matvecs_fp32, res=info.rel_residual, E=E)

    # warmup
    for _ in range(args.warmup):
        h, x, st = run(F.MIXED, True)
        h.close()
        log("warmup step %.0f ms" % st["total_ms"])
    torch.cuda.synchronize()
    # timed steps: the whole path, mixed precision
    prof_tot = {k: [0.0, 0.0] for k in ("ms_total", "ms_near", "ms_up", "ms_m2l", "ms_down")}
    mv = [0, 0]
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h, x, st = run(F.MIXED, True)
        p = h.profile()
        for k in prof_tot:
            for j in range(2):
                prof_tot[k][j] += p[k][j]
        for j in range(2):
            mv[j] += p["matvecs"][j]
        steps.append(st)
        ti = h.tree_info()
        flops_m2l = m2l_flops(h)
        near_pairs = ti.near_pairs
        E_mixed = st["E"]
        h.close()
        log("timed step %.0f ms (%d inner iterations)" % (st["total_ms"], st["iters"]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    # mixed operator throughput (FP32 matvecs dominate; FP64 outer ones reported too)
    mv32_ms = prof_tot["ms_total"][1] / max(mv[1], 1)
    mv64_in_mixed_ms = prof_tot["ms_total"][0] / max(mv[0], 1)
    value = N / (mv32_ms * 1e-3) / 1e6
    # FP64 reference path (outside the timed region)
    h64, x64, st64 = run(F.FP64, True)
    p64 = h64.profile()
    mv64_ms = p64["ms_total"][0] / max(p64["matvecs"][0], 1)
    # the direct energy sum of the FP64 solution (the treecode energy's reference)
    torch.cuda.synchronize()
    t = time.perf_counter()
    E64_direct = h64.solvation_energy(x64, w["xq"], w["q"])
    direct_ms = 1e3 * (time.perf_counter() - t)
    h64.close()
    # reference: FP64 with the direct right-hand side and the direct energy sum
    href, _, stref = run(F.FP64, False, direct=True)
    href.close()
    E_ref = stref["E"]
    log("fp64 reference (direct sums) %.0f ms" % stref["total_ms"])
    log("fp64 path %.0f ms (%d iterations)" % (st64["total_ms"], st64["iters"]))
    # dominant single kernel of the mixed matvec: the near-field block SpMV
    # (its launch is exactly the "near" interval of the profile events; it
    # runs beside the far field on a second stream, so this is its duration
    # in the path).  The other phase intervals overlap and are reported as
    # measured (up: upward pass with the finest MtL levels beside it; m2l: the
    # rest of MtL until the join; down: LtL and LtP).
    phases = {k: prof_tot[k][1] / max(mv[1], 1) for k in ("ms_near", "ms_up", "ms_m2l", "ms_down")}
    spmv_bytes = near_pairs * 16 + 2 * N * 8 + 2 * N * 8
    ach = spmv_bytes / (phases["ms_near"] * 1e-3) / 1e9
    roof = {"kernel": "k_spmv<float4> (near-field block SpMV, one launch per matvec)", "bound": "hbm",
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": TRAFFIC_SPMV, "avg_launch_ms": phases["ms_near"],
            "algorithmic_bytes_per_launch": spmv_bytes}
    line = {
        "metric": METRIC, "value": value, "unit": "Mpanels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operator, f64 accumulation/Krylov", "data": "synthetic",
        "config": {"workload": "%s: Gaussian isosurface of 20,000 packed atoms, %d panels, "
                               "%d charges, eps 1/80, kappa 0.1257" % (args.workload, N, len(w["q"])),
                   **{k: v for k, v in PARAMS.items()}},
        "roofline": roof,
        "matvec_ms": {"mixed_fp32": mv32_ms, "fp64": mv64_ms,
                      "mixed_phases": phases,
                      "fp64_phases": {k: p64[k][0] / max(p64["matvecs"][0], 1)
                                      for k in ("ms_near", "ms_up", "ms_m2l", "ms_down")}},
        "matvec_mpanels_fp64": N / (mv64_ms * 1e-3) / 1e6,
        "m2l_flops_per_matvec": flops_m2l, "near_pairs": near_pairs,
        "time_to_solve_ms": {"mixed": float(np.median([s["total_ms"] for s in steps])),
                             "fp64": st64["total_ms"]},
        "solve_breakdown_mixed": steps[-1], "solve_breakdown_fp64": st64,
        "energy_kcal": {"mixed": E_mixed, "fp64": st64["E"],
                        "rel_diff": abs(E_mixed - st64["E"]) / abs(st64["E"]),
                        "method": "right-hand side and energy by the Cartesian treecode, theta %.2f / %.2f, "
                                  "FMM moments and locals, orders min(p_l, %d)" % (PARAMS["rhs_theta"], ENERGY_THETA,
                                                                                   ENERGY_PMAX),
                        "fp64_energy_direct_sum": E64_direct, "energy_direct_sum_ms": direct_ms,
                        "treecode_energy_vs_direct_fp64": abs(st64["E"] - E64_direct) / abs(E64_direct),
                        "fp64_reference_direct_rhs_and_energy": E_ref,
                        "reference_time_to_solve_ms": stref["total_ms"],
                        "reference_rhs_ms": stref["t_rhs_ms"],
                        "mixed_vs_reference": abs(E_mixed - E_ref) / abs(E_ref),
                        "fp64_vs_reference": abs(st64["E"] - E_ref) / abs(E_ref)},
        "mlp": dict(mlp_info, gate_tol=MLP_GATE,
                    gated_pairs=steps[-1]["mlp_gated"], candidate_pairs=steps[-1]["mlp_candidates"],
                    note="mixed path = FP32 operator with the gated surrogate near field inside FP64 "
                         "flexible GMRES; the FP64 path uses cubature for every pair; energy rel_diff "
                         "is the error of mixed+MLP against the FP64 path"),
    }
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = 2 * a.numel() * 8
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_rows)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
