"""Benchmark of the Galerkin BIE Poisson-Boltzmann hot path on one MI355X.

One step = one full pass of the path on the ~500k-panel workload: cluster
tree, near-field assembly (singular cubature, near-singular pairs replaced by
the learned surrogate where its calibrated error passes the stated gate) with
preconditioner factors, right-hand side, mixed-precision flexible GMRES to a
1e-6 true residual of that operator (FP32 FMM/near field inside, FP64
outside), and the solvation energy.  The surrogate is trained once before the
timed steps (time reported separately).  Inputs (mesh, charges) are host
arrays handed to the library, as its C ABI defines.

value = FMM matvec throughput [Mpanels/s] of the mixed-precision operator,
from HIP events around every matvec issued inside the timed steps.  The same
line reports the GMRES time-to-1e-6 of the mixed path with and without the
surrogate and of the plain FP64 path, the operator and solution errors of the
mixed paths against the FP64 cubature operator, the dominant kernel against
its roofline (and the other large one), secondary workloads, and the FP64 CPU
oracle's FMM matvec timed on the host.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM matvec Mpanels/s + GMRES time-to-1e-6 (mixed+MLP vs FP64) at 500k panels"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (and FP32 matrix) peak
FP64_PEAK_TFLOPS = 78.6
# acceptance parameter of the treecode energy (rho_l / R <= theta) and its
# order cap (terms |b| <= min(p_l, 6))
ENERGY_THETA = 0.5
ENERGY_PMAX = 6
# HBM traffic per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated with a
# device copy) is read from these summaries; each names the sha256 of the
# kernel source it was measured on, and a changed source makes it null
TRAFFIC_FILES = {"k_spmv": "profiles/k_spmv_ellipsoid500k_hbm_traffic.md",
                 "k_m2l_leaf": "profiles/k_m2l_leaf_ellipsoid500k_hbm_traffic.md"}
KERNEL_SOURCE = "paper_2110_13778_amd/csrc/fmm.hip"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoid500k")
    ap.add_argument("--fp64-runs", type=int, default=5, help="FP64 path solves (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads (kirkwood2, globule200k, ellipsoid1m)")
    ap.add_argument("--cpu-solve", action="store_true",
                    help="only the oracle's whole solve on the 81,920-panel multi-charge sphere on the host "
                         "(about half an hour of one core; no GPU), printed as one JSON line")
    ap.add_argument("--mlp-epochs", type=int, default=240,
                    help="training epochs of the near-field surrogate (before the timed steps)")
    ap.add_argument("--mlp-pairs", type=int, default=2000000,
                    help="training pairs drawn per training mesh (two meshes; the default takes every "
                         "near-singular pair of both)")
    ap.add_argument("--no-hat", action="store_true",
                    help="skip the continuous piecewise-linear (hat-function) leg on the main workload")
    ap.add_argument("--hat-only", action="store_true",
                    help="run only the hat-function leg (for per-kernel profiles of that path) and print it")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


PARAMS = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8, quad_duffy=7,
              near_ratio=2.0, tol=1e-6, max_iter=200, max_outer=5, inner_tol=5e-7,
              precond=3,   # block-diagonal preconditioner over consecutive leaves, <= 32 panels
              rhs_theta=0.5, rhs_pmax=6)   # right-hand side by the reverse treecode
MLP_GATE = 0.05         # stated per-pair error tolerance of the gated near field


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def hat_leg(F, torch, w, dev, E_box_ref, runs=3):
    """The continuous piecewise-linear basis (hat functions at the vertices) on
    the same workload and tree: FP32-inner flexible GMRES and FP64 GMRES with
    the Jacobi preconditioner, right-hand side and energy by the treecodes as
    in the box-function step.  Median of `runs` whole solves per precision
    (build, assembly, solve, energy), with the per-matvec phase times of the
    median run; the energy of the last FP64 solve also by the direct sum."""
    N, V = len(w["tris"]), len(w["verts"])
    prm = dict(PARAMS, precond=F.PRECOND_DIAG, max_iter=300)
    out = {"panels": N, "vertices": V, "precond": "Jacobi (the diagonal of A)",
           "rhs_and_energy": "treecodes, theta %.2f / %.2f, order cap %d / %d" % (
               PARAMS["rhs_theta"], ENERGY_THETA, PARAMS["rhs_pmax"], ENERGY_PMAX)}
    near_pairs = hat_rows = hat_entries = 0
    E_direct = None
    for tag, prec in (("mixed", F.MIXED), ("fp64", F.FP64)):
        sts = []
        p = 1 if prec == F.MIXED else 0
        for _ in range(runs):
            h = F.Handle(precision=prec, eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"],
                         basis=F.BASIS_S1, **prm)
            h.set_profiling(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.build_tree(w["verts"], w["tris"])
            t1 = time.perf_counter()
            h.assemble_nearfield()
            t2 = time.perf_counter()
            x = torch.zeros(2 * V, dtype=torch.float64, device=dev)
            code, info = h.solve(w["xq"], w["q"], x)
            t3 = time.perf_counter()
            E = h.solvation_energy_treecode(x, w["xq"], w["q"], ENERGY_THETA, p_max=ENERGY_PMAX)
            t4 = time.perf_counter()
            if prec == F.FP64:
                E_direct = h.solvation_energy(x, w["xq"], w["q"])
            pr = h.profile()
            ti = h.tree_info()
            near_pairs, hat_rows, hat_entries = ti.near_pairs, ti.hat_rows, ti.hat_entries
            mv = max(pr["matvecs"][p], 1)
            sts.append(dict(code=code, total_ms=1e3 * (t4 - t0), tree_ms=1e3 * (t1 - t0),
                            assemble_ms=1e3 * (t2 - t1), solve_ms=1e3 * (t3 - t2), energy_ms=1e3 * (t4 - t3),
                            t_rhs_ms=info.t_rhs_ms, t_iterations_ms=info.t_solve_ms,
                            iters=info.inner_iterations, outer=info.outer_iterations, res=info.rel_residual, E=E,
                            setup_stages_ms={k: pr[k] for k in ("ms_tree", "ms_classify", "ms_singular",
                                                                "ms_fmm_setup", "ms_precond")},
                            matvec_ms=pr["ms_total"][p] / mv, spmv_ms=pr["ms_near"][p] / mv,
                            m2l_leaf_ms=pr["ms_m2l_leaf"][p] / mv, matvecs=pr["matvecs"][p]))
            h.close()
        out[tag] = sts[int(np.argsort([s["total_ms"] for s in sts])[len(sts) // 2])]
        out[tag]["total_ms_runs"] = [s["total_ms"] for s in sts]
        log("hat basis %s: %.0f ms to 1e-6 (%d inner iterations), matvec %.3f ms"
            % (tag, out[tag]["total_ms"], out[tag]["iters"], out[tag]["matvec_ms"]))
    # the near-field SpMV over vertex pairs: one FP32 entry quadruple per
    # (leaf row vertex, source vertex), every vertex's (phi, dphi) read once and
    # the two results of every row written
    spmv_bytes = hat_entries * 16 + V * 16 + hat_rows * 16
    ach = spmv_bytes / (out["mixed"]["spmv_ms"] * 1e-3) / 1e9
    out["near_field"] = {"stored_panel_pairs": near_pairs, "vertex_pair_rows": hat_rows,
                         "vertex_pair_entries": hat_entries, "corner_pair_entries": 9 * near_pairs}
    out["spmv_fp32"] = {"kernel": "k_spmv<float4> over vertex pairs (one launch per matvec)", "bound": "hbm",
                        "avg_launch_ms": out["mixed"]["spmv_ms"], "algorithmic_bytes_per_launch": spmv_bytes,
                        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}
    out["matvec_mvertices_per_s"] = {"mixed_fp32": V / (out["mixed"]["matvec_ms"] * 1e-3) / 1e6,
                                     "fp64": V / (out["fp64"]["matvec_ms"] * 1e-3) / 1e6}
    E64, Em = out["fp64"]["E"], out["mixed"]["E"]
    out["energy_kcal"] = {"mixed": Em, "fp64": E64, "mixed_vs_fp64": abs(Em - E64) / abs(E64),
                          "fp64_direct_sum": E_direct, "treecode_vs_direct": abs(E64 - E_direct) / abs(E_direct),
                          "box_fp64_direct_sums": E_box_ref,
                          "hat_vs_box": None if E_box_ref is None else abs(E_direct - E_box_ref) / abs(E_box_ref)}
    return out


def sha256(path):
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, or None when
    the summary is missing or was measured on another kernel source."""
    path = os.path.join(ROOT, TRAFFIC_FILES[kernel])
    if not os.path.exists(path):
        return None, "no counter summary"
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)", txt)
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not m or not h:
        return None, "summary without traffic/source lines"
    if h.group(1) != sha256(KERNEL_SOURCE):
        return None, "kernel source changed since the counters were taken"
    return int(m.group(1)), TRAFFIC_FILES[kernel]


def train_surrogate(F, torch, pairs_per_mesh, epochs):
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
    torch.cuda.synchronize()
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


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(w, prm):
    """The FP64 oracle's FMM matvec (oracle.fmm, numpy with its BLAS threads)
    on the benchmark mesh and tree.  Timed at full size: the near-field
    product (the oracle's stored-entry product over the 74M stored pairs of
    the tree's neighbour lists; entry values are random, the product's cost
    does not depend on them), the upward pass, the downward pass and the
    evaluation.  The interaction phase (MtL) is timed on a random sample of
    target clusters per level (all clusters of levels with at most 256) and
    scaled by the level's pairs over the sampled pairs.  Setup (tree, panel
    moments, the pair lists) is not timed, as on the GPU."""
    from oracle import fmm as ofmm
    from oracle import tree as otree
    from oracle.geometry import panels
    P = panels(w["verts"], w["tris"])
    N = P.n
    eps = w["eps_out"] / w["eps_in"]
    tr = otree.build(P, prm["leaf_size"], prm["eta0"])
    O = ofmm.setup(P, tr, eps, w["kappa"], p_leaf=prm["p_leaf"], adaptive=prm["adaptive"],
                   p_max=prm["p_max"], with_near=False)
    leaf = tr.levels[tr.L]
    ii, jj = [], []
    for c in range(leaf.n):
        tgt = tr.perm[leaf.start[c]:leaf.end[c]]
        src = np.concatenate([tr.perm[leaf.start[c2]:leaf.end[c2]] for c2 in leaf.nbr[c]])
        ii.append(np.repeat(tgt, len(src)))
        jj.append(np.tile(src, len(tgt)))
    rng = np.random.default_rng(7)
    O.near_i, O.near_j = np.concatenate(ii), np.concatenate(jj)
    del ii, jj
    O.near_B = rng.standard_normal((len(O.near_i), 4))
    x = rng.standard_normal(2 * N)
    phi, dphi = x[:N], x[N:]
    t = {}
    c0 = time.process_time()
    t0 = time.perf_counter()
    ofmm.matvec(O, x, far=False)
    t["near"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    M0, Mk = ofmm.upward(O, phi, dphi)
    t["upward"] = time.perf_counter() - t0
    lam0, lamk, m2l, m2l_wall, sampled = {}, {}, 0.0, 0.0, {}
    for l in range(tr.lmin, tr.L + 1):
        cl = tr.levels[l]
        sel = np.arange(cl.n) if cl.n <= 256 else np.sort(rng.choice(cl.n, 256, replace=False))
        pairs_all = sum(len(s) for s in cl.inter)
        pairs_sel = sum(len(cl.inter[c]) for c in sel)
        t0 = time.perf_counter()
        lam0[l], lamk[l] = ofmm.interaction(O, M0, Mk, l, sel)
        dt = time.perf_counter() - t0
        m2l_wall += dt
        m2l += dt * pairs_all / max(pairs_sel, 1)
        sampled[l] = [int(len(sel)), int(cl.n), int(pairs_sel), int(pairs_all)]
    t["m2l_scaled"] = m2l
    t0 = time.perf_counter()
    ofmm.downward(O, lam0, tr.lmin)
    ofmm.downward(O, lamk, tr.lmin)
    ofmm.evaluate(O, lam0[tr.L], lamk[tr.L])
    t["downward_evaluate"] = time.perf_counter() - t0
    cpu = time.process_time() - c0
    wall = sum(v for k, v in t.items() if k != "m2l_scaled") + m2l_wall
    total = sum(t.values())
    model, ncpu, avail = host_cpu()
    return {"value": N / total / 1e6, "unit": "Mpanels/s",
            "cores": avail, "kind": "oracle",
            "sample": "oracle.fmm matvec on the benchmark mesh (%d panels, same tree, orders and near "
                      "pairs): near-field product, upward pass, downward pass and evaluation timed at full "
                      "size; MtL timed on up to 256 random target clusters per level and scaled by pairs "
                      "(level: [sampled, clusters, sampled pairs, pairs] = %s); numpy/BLAS on the host's "
                      "threads" % (N, json.dumps(sampled)),
            "cpu_model": model, "nproc": ncpu, "threads_available": avail,
            "effective_parallelism": cpu / wall,
            "matvec_s": total, "stage_s": t, "timed_wall_s": wall,
            "process_cpu_s": cpu}


def cpu_fmm_c2():
    """The oracle's whole FMM far field (no sampling) on the 81,920-panel
    sphere (adaptive orders 3..8, leaf 32)."""
    from oracle import fmm as ofmm
    from oracle import tree as otree
    from oracle.geometry import panels
    from synth import workload
    w = workload("kirkwood2")
    P = panels(w["verts"], w["tris"])
    tr = otree.build(P, 32, 0.8)
    O = ofmm.setup(P, tr, w["eps_out"] / w["eps_in"], w["kappa"], p_leaf=3, adaptive=1, p_max=8,
                   with_near=False)
    x = np.random.default_rng(8).standard_normal(2 * P.n)
    c0 = time.process_time()
    t0 = time.perf_counter()
    ofmm.far_field(O, x[:P.n], x[P.n:])
    dt = time.perf_counter() - t0
    return {"workload": "kirkwood2 (81,920 panels)", "far_field_s": dt,
            "process_cpu_s": time.process_time() - c0, "mpanels_per_s_far_field_only": P.n / dt / 1e6}


def cpu_solve_c2():
    """The FP64 oracle's whole solve on the 81,920-panel multi-charge sphere
    as it stands: tree, FMM setup with the near field (every stored pair by
    its cubature rule), block preconditioner, right-hand side, right-
    preconditioned GMRES to 1e-6 with the oracle's FMM matvec (adaptive orders
    3..8, leaf 32, eta0 0.8), direct energy sum.  One process."""
    from oracle import fmm as ofmm
    from oracle import solve as osolve
    from oracle import tree as otree
    from oracle.geometry import panels
    from synth import workload
    w = workload("kirkwood2")
    P = panels(w["verts"], w["tris"])
    eps = w["eps_out"] / w["eps_in"]
    t = {}
    c0 = time.process_time()
    t0 = time.perf_counter()
    tr = otree.build(P, 32, 0.8)
    t["tree"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    F = ofmm.setup(P, tr, eps, w["kappa"], p_leaf=3, adaptive=True, p_max=8)
    t["fmm_setup_and_near_field"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    M = osolve.block_preconditioner(P, tr, eps, w["kappa"])
    t["preconditioner"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = osolve.rhs(P, w["xq"], w["q"], w["eps_in"])
    t["rhs"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, its, hist = osolve.gmres(lambda z: ofmm.matvec(F, z), b, tol=1e-6, max_iter=100, precond=M)
    t["gmres"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    E = osolve.energy(P, x, w["xq"], w["q"], eps, w["kappa"])
    t["energy"] = time.perf_counter() - t0
    model, ncpu, avail = host_cpu()
    total = sum(t.values())
    return {"workload": "kirkwood2: 81,920-panel sphere, 50 charges", "kind": "oracle",
            "time_to_solve_s": total, "stage_s": t, "gmres_iterations": int(its),
            "estimated_residual": float(hist[-1]), "energy_kcal": float(E), "near_pairs": int(len(F.near_i)),
            "process_cpu_s": time.process_time() - c0, "cpu_model": model, "nproc": ncpu,
            "threads_available": avail}


def main():
    args = parse()
    if args.cpu_solve:
        print(json.dumps({"cpu_baseline_solve": cpu_solve_c2()}))
        return
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

    log("workload %s: %d panels, %d charges" % (args.workload, N, len(w["q"])))
    if args.hat_only:
        print(json.dumps({"workload": args.workload, "hat_basis": hat_leg(F, torch, w, dev, None)}))
        return
    blob, mlp_info = train_surrogate(F, torch, args.mlp_pairs, args.mlp_epochs)
    log("surrogate trained on %d pairs in %.1f s" % (mlp_info["pairs"], mlp_info["train_s"]))

    def run(w, prec, profile, mlp=True, direct=False, keep=False):
        N = len(w["tris"])
        extra = dict(mlp_mode=F.MLP_GATED, mlp_gate_tol=MLP_GATE) if (prec == F.MIXED and mlp) else {}
        prm = dict(PARAMS, rhs_theta=0.0) if direct else PARAMS
        h = F.Handle(precision=prec, eps_in=w["eps_in"], eps_out=w["eps_out"],
                     kappa=w["kappa"], **prm, **extra)
        if extra:
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
        gated = h.mlp_stats() if extra else (0, 0)
        pr = h.profile()
        setup = {k: pr[k] for k in ("ms_tree", "ms_classify", "ms_surrogate", "ms_singular", "ms_fmm_setup",
                                    "ms_precond")}
        st = dict(code=code, mlp_gated=gated[0], mlp_candidates=gated[1], setup_stages_ms=setup,
                  t_rhs_ms=info.t_rhs_ms, t_iterations_ms=info.t_solve_ms, tree_ms=1e3 * (t1 - t0),
                  assemble_ms=1e3 * (t2 - t1), solve_ms=1e3 * (t3 - t2), energy_ms=1e3 * (t4 - t3),
                  total_ms=1e3 * (t4 - t0), iters=info.inner_iterations,
                  outer=info.outer_iterations, mv64=info.matvecs_fp64,
                  mv32=info.matvecs_fp32, res=info.rel_residual, E=E)
        if not keep:
            h.close()
            return None, None, st
        return h, x, st

    # warmup
    for _ in range(args.warmup):
        _, _, st = run(w, F.MIXED, True)
        log("warmup step %.0f ms" % st["total_ms"])
    torch.cuda.synchronize()
    # timed steps: the whole path, mixed precision with the gated surrogate
    prof_tot = {k: [0.0, 0.0] for k in ("ms_total", "ms_near", "ms_up", "ms_m2l", "ms_down", "ms_m2l_leaf")}
    mv = [0, 0]
    steps = []
    h_mix = x_mix = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        last = k == args.steps - 1
        h, x, st = run(w, F.MIXED, True, keep=last)
        if last:
            h_mix, x_mix = h, x
            p = h.profile()
            ti = h.tree_info()
        steps.append(st)
        log("timed step %.0f ms (%d inner iterations)" % (st["total_ms"], st["iters"]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    # per-matvec phase times of the last timed step (the same operator every step)
    for k in prof_tot:
        for j in range(2):
            prof_tot[k][j] += p[k][j]
    for j in range(2):
        mv[j] += p["matvecs"][j]
    near_pairs = ti.near_pairs
    E_mixed = steps[-1]["E"]
    mv32_ms = prof_tot["ms_total"][1] / max(mv[1], 1)
    value = N / (mv32_ms * 1e-3) / 1e6
    # plain FP64 path (cubature everywhere, FP64 GMRES): median of several solves
    runs64 = []
    h64 = x64 = None
    for k in range(args.fp64_runs):
        last = k == args.fp64_runs - 1
        h, x, st = run(w, F.FP64, True, keep=last)
        runs64.append(st)
        if last:
            h64, x64 = h, x
    order = np.argsort([s["total_ms"] for s in runs64])
    st64 = runs64[order[len(order) // 2]]
    p64 = h64.profile()
    mv64_ms = p64["ms_total"][0] / max(p64["matvecs"][0], 1)
    log("fp64 path %.0f ms median of %d (%d iterations)" % (st64["total_ms"], len(runs64), st64["iters"]))
    # mixed precision without the surrogate (cubature everywhere)
    runs_nm = []
    h_nm = None
    for k in range(3):
        h, x, st = run(w, F.MIXED, True, mlp=False, keep=(k == 2))
        runs_nm.append(st)
        if k == 2:
            h_nm = h
    st_nm = runs_nm[int(np.argsort([s["total_ms"] for s in runs_nm])[1])]
    log("mixed without surrogate %.0f ms (%d inner iterations)" % (st_nm["total_ms"], st_nm["iters"]))
    # operator and solution errors against the FP64 cubature operator
    rng = np.random.default_rng(11)
    xr = torch.tensor(rng.standard_normal(2 * N), dtype=torch.float64, device=dev)
    y64 = torch.empty_like(xr)
    yt = torch.empty_like(xr)
    h64.matvec(xr, y64, F.FP64)

    def rel_to_64(hh, prec):
        hh.matvec(xr, yt, prec)
        return float(torch.linalg.norm(yt - y64) / torch.linalg.norm(y64))

    op_err = {"mixed_fp32_with_surrogate": rel_to_64(h_mix, F.MIXED),
              "fp64_with_surrogate_entries": rel_to_64(h_mix, F.FP64),
              "mixed_fp32_without_surrogate": rel_to_64(h_nm, F.MIXED)}
    b64 = torch.empty_like(xr)
    h64.rhs_treecode(w["xq"], w["q"], PARAMS["rhs_theta"], b64, p_max=PARAMS["rhs_pmax"])
    h64.matvec(x_mix, yt, F.FP64)
    res_true = float(torch.linalg.norm(b64 - yt) / torch.linalg.norm(b64))
    h_nm.close()
    # the direct energy sum of the FP64 solution (the treecode energy's reference)
    torch.cuda.synchronize()
    t = time.perf_counter()
    E64_direct = h64.solvation_energy(x64, w["xq"], w["q"])
    direct_ms = 1e3 * (time.perf_counter() - t)
    h64.close()
    h_mix.close()
    # reference: FP64 with the direct right-hand side and the direct energy sum
    _, _, stref = run(w, F.FP64, False, direct=True)
    E_ref = stref["E"]
    log("fp64 reference (direct sums) %.0f ms" % stref["total_ms"])
    # dominant kernels of the mixed matvec: the near-field block SpMV (its
    # launch is exactly the "near" interval of the profile events) and the
    # leaf level's MtL (events around its launch on its own stream); both run
    # beside other kernels, so these are durations in the path
    phases = {k: prof_tot[k][1] / max(mv[1], 1) for k in ("ms_near", "ms_up", "ms_m2l", "ms_down",
                                                           "ms_m2l_leaf")}
    spmv_bytes = near_pairs * 16 + 2 * N * 8 + 2 * N * 8
    ach = spmv_bytes / (phases["ms_near"] * 1e-3) / 1e9
    tr_spmv, tr_spmv_src = measured_traffic("k_spmv")
    roof_spmv = {"kernel": "k_spmv<float4> (near-field block SpMV, one launch per matvec)", "bound": "hbm",
                 "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                 "traffic": tr_spmv, "traffic_source": tr_spmv_src, "avg_launch_ms": phases["ms_near"],
                 "algorithmic_bytes_per_launch": spmv_bytes}
    L = ti.levels
    pL = ti.lev_order[L]
    from math import comb
    m2l_leaf_flops = ti.lev_pairs[L] * 2 * 2 * comb(pL + 6, 6)
    ach_m2l = m2l_leaf_flops / (phases["ms_m2l_leaf"] * 1e-3) / 1e12
    tr_m2l, tr_m2l_src = measured_traffic("k_m2l_leaf")
    roof_m2l = {"kernel": "leaf-level MtL (order %d, %d cluster pairs, FP32, one launch per matvec)"
                          % (pL, ti.lev_pairs[L]),
                "bound": "alu", "achieved": ach_m2l, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": ach_m2l / FP32_PEAK_TFLOPS, "traffic": tr_m2l, "traffic_source": tr_m2l_src,
                "avg_launch_ms": phases["ms_m2l_leaf"], "algorithmic_flops_per_launch": m2l_leaf_flops}
    if phases["ms_m2l_leaf"] >= phases["ms_near"]:
        roof, roof_other = roof_m2l, roof_spmv
    else:
        roof, roof_other = roof_spmv, roof_m2l
    med = lambda xs: float(np.median(xs))
    line = {
        "metric": METRIC, "value": value, "unit": "Mpanels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 operator, f64 accumulation/Krylov", "data": "synthetic",
        "config": {"workload": "%s: Gaussian isosurface of 20,000 packed atoms, %d panels, "
                               "%d charges, eps 1/80, kappa 0.1257" % (args.workload, N, len(w["q"])),
                   **{k: v for k, v in PARAMS.items()}},
        "roofline": roof,
        "roofline_other": [roof_other],
        "matvec_ms": {"mixed_fp32": mv32_ms, "fp64": mv64_ms,
                      "mixed_phases": phases,
                      "fp64_phases": {k: p64[k][0] / max(p64["matvecs"][0], 1)
                                      for k in ("ms_near", "ms_up", "ms_m2l", "ms_down", "ms_m2l_leaf")}},
        "matvec_mpanels_fp64": N / (mv64_ms * 1e-3) / 1e6,
        "m2l_flops_per_matvec": 2.0 * ti.m2l_flops_fp, "near_pairs": near_pairs,
        "time_to_solve_ms": {"mixed_with_surrogate": med([s["total_ms"] for s in steps]),
                             "mixed_without_surrogate": st_nm["total_ms"],
                             "fp64": st64["total_ms"],
                             "fp64_runs": [s["total_ms"] for s in runs64],
                             "mixed_without_surrogate_runs": [s["total_ms"] for s in runs_nm]},
        "solve_breakdown_mixed": steps[-1], "solve_breakdown_mixed_without_surrogate": st_nm,
        "solve_breakdown_fp64": st64,
        "errors_vs_fp64_cubature": {
            "operator_rel_l2": op_err,
            "mixed_with_surrogate_solution_true_residual": res_true,
            "note": "operator: ||A' x - A64 x|| / ||A64 x|| for a random x, A64 the FP64 cubature operator; "
                    "residual: ||b - A64 x_mixed|| / ||b|| of the mixed+surrogate solution (same treecode b)"},
        "energy_kcal": {"mixed": E_mixed, "mixed_without_surrogate": st_nm["E"], "fp64": st64["E"],
                        "rel_diff": abs(E_mixed - st64["E"]) / abs(st64["E"]),
                        "rel_diff_without_surrogate": abs(st_nm["E"] - st64["E"]) / abs(st64["E"]),
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
                    assembly_ms_with_surrogate=steps[-1]["assemble_ms"],
                    assembly_ms_without_surrogate=st_nm["assemble_ms"],
                    inner_iterations_with_surrogate=steps[-1]["iters"],
                    inner_iterations_without_surrogate=st_nm["iters"],
                    note="mixed path = FP32 operator with the gated surrogate near field inside FP64 "
                         "flexible GMRES; the FP64 path uses cubature for every pair; energy rel_diff "
                         "is the error of mixed+MLP against the FP64 path"),
    }
    if not args.no_secondary:
        sec = {}
        for name in ("kirkwood2", "globule200k", "ellipsoid1m"):
            w2 = workload(name)
            r = {"panels": len(w2["tris"]), "charges": len(w2["q"])}
            for tag, prec, mlp in (("mixed_with_surrogate", F.MIXED, True), ("fp64", F.FP64, True)):
                _, _, s2 = run(w2, prec, True, mlp=mlp)
                r[tag] = {k: s2[k] for k in ("total_ms", "assemble_ms", "solve_ms", "iters", "outer", "res", "E")}
            r["energy_rel_diff"] = abs(r["mixed_with_surrogate"]["E"] - r["fp64"]["E"]) / abs(r["fp64"]["E"])
            sec[name] = r
            log("secondary %s: %d panels, mixed %.0f ms, fp64 %.0f ms" % (
                name, r["panels"], r["mixed_with_surrogate"]["total_ms"], r["fp64"]["total_ms"]))
        line["secondary_workloads"] = sec
    if not args.no_hat:
        line["hat_basis"] = hat_leg(F, torch, w, dev, E_ref)
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = 2 * a.numel() * 8
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle FMM on the host)")
        line["cpu_baseline"] = cpu_baseline(w, PARAMS)
        line["cpu_baseline"]["c2_full_far_field"] = cpu_fmm_c2()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
