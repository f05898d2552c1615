"""Throughput of boundary-MPS environments on one MI355X.

One step = one complete environment of the 8x8, D=4, chi=32 near-product
PEPS (top and bottom boundaries by ALS row absorption, then the norm, 64
<S^z> and 112 Heisenberg bond energies from the one- and two-row
sandwiches), inputs resident in HBM: `value` is environments/s of that step
in FP64.  The same JSON line carries the other workloads of the benchmark
set, each with its error against the FP64 path: the 10x10 D=6 chi=72 lattice
in FP64/FP32/BF16, the 256 cluster windows per n of a 16x16 D=6 lattice in
FP32 and FP64, a subset of the 32 batched instances (all D <= 5 ones and the
smallest D = 8 one) in FP64 and BF16; the ALS convergence of the truncation;
the roofline of the dominant contraction kernel; the oracle on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
                    [--no-workloads] [--workloads convergence,evolution]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}   # dense MFMA TFLOP/s, MI355X
HBM_TBS = 8.0                                          # HBM3E, TB/s
WORKLOAD_TAG = "env_8x8_D4_chi32_f64"


def kernel_slug(name):
    """File-name form of a kernel variant: runs of other characters become one '_'."""
    import re
    return re.sub(r"[^0-9A-Za-z]+", "_", name).strip("_")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` on this workload from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy of
    known size); None when there is none or the kernel or recorder source
    changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_slug(kernel)}__{WORKLOAD_TAG}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    # the kernel's source and the recorder's, which fixes its launch shapes
    for name in ("kernels.hip", "runtime.cpp"):
        src = os.path.join(ROOT, "paper_1311_6696_amd", "csrc", name)
        if fields.get(f"{name} sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
    if "traffic bytes per launch" not in fields:
        return None
    return float(fields["traffic bytes per launch"])
def run_steps(sess, dev_state, chi, dtype, halfsweeps, n, split=None, columns=False):
    """n full environments; `split` (a list) receives (boundary_s, expect_s) per step.
    columns: vertical bonds from the left/right boundaries instead of two-row sandwiches."""
    res = None
    for _ in range(n):
        t0 = time.perf_counter()
        envs = sess.env_boundary([dev_state], chi, dtype, halfsweeps, columns=columns)
        t1 = time.perf_counter()
        res = sess.expect(envs)[0]
        t2 = time.perf_counter()
        if split is not None:
            split.append((t1 - t0, t2 - t1))
        for e in envs:
            e.free()
    return res


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def energy(r):
    return float(np.sum(r["bond_h"]) + np.sum(r["bond_v"]))


def timed(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) / reps


def max_bond_diff(a, b):
    return float(max(np.max(np.abs(a["bond_h"] - b["bond_h"])), np.max(np.abs(a["bond_v"] - b["bond_v"]))))


def als_convergence(sess, st, chi, res_h4, H=4):
    """How far the default ALS truncation (H half-sweeps from a random start)
    is from its fixed point: the largest relative change of the squared centre
    norm in the last half-sweep over all truncated rows, and the largest
    change of any bond energy and <S^z> when the rows run 2H and 4H
    half-sweeps instead."""
    env = sess.env_boundary([st], chi, "f64", H)[0]
    w = env.info()
    env.free()
    rel = np.abs(w[:, -1] - w[:, -2]) / np.abs(w[:, -1]) if w.shape[1] > 1 else np.array([np.nan])
    out = {"halfsweeps": H, "truncated_rows": int(w.shape[0]),
           "max_rel_omega_change_last_halfsweep": float(np.max(rel))}
    for HH in (2 * H, 4 * H):
        r = run_steps(sess, st, chi, "f64", HH, 1)
        out[f"max_bond_change_H{H}_vs_H{HH}"] = max_bond_diff(res_h4, r)
        out[f"max_sz_change_H{H}_vs_H{HH}"] = float(np.max(np.abs(res_h4["sz"] - r["sz"])))
    return out


def side_precision(sess, binding, torch):
    """10x10, D=6, unit-norm Gaussian sites, chi=72: one full environment per
    dtype; errors are against the FP64 GPU path (itself checked against the
    oracle at this shape on the boundaries of rows 0-2 and at smaller sizes)."""
    from paper_1311_6696_amd.inputs import WORKLOADS, workload_peps
    cfg = WORKLOADS["10x10_D6_chi72"]
    st = binding.to_device(workload_peps("10x10_D6_chi72"))
    out, ref = {}, None
    for dt in ("f64", "f32", "bf16"):
        note(f"10x10 D=6 chi=72 {dt}")
        run = lambda: run_steps(sess, st, cfg["chi"], dt, 4, 1)
        run()   # warm-up (allocations)
        r, t = timed(torch, run, 2)
        if ref is None:
            ref = r
        e, e0 = energy(r), energy(ref)
        out[dt] = {"env_per_s": 1.0 / t, "s_per_env": t, "tflops": r["flops"] / t / 1e12,
                   "pct_peak": 100.0 * r["flops"] / t / 1e12 / PEAK[dt], "tflop_per_env": r["flops"] / 1e12,
                   "rel_energy_err_vs_f64": abs(e - e0) / abs(e0),
                   "max_bond_err_vs_f64": max_bond_diff(r, ref)}
        out[dt]["speedup_vs_f64"] = out["f64"]["s_per_env"] / t
    # FP64 with the vertical bonds from the column boundaries
    note("10x10 D=6 chi=72 f64 with column boundaries")
    run = lambda: run_steps(sess, st, cfg["chi"], "f64", 4, 1, columns=True)
    run()
    r, t = timed(torch, run, 2)
    out["f64_columns"] = {"env_per_s": 1.0 / t, "s_per_env": t, "tflop_per_env": r["flops"] / 1e12,
                          "speedup_vs_f64": out["f64"]["s_per_env"] / t,
                          "max_bond_v_gap_vs_two_row": float(np.max(np.abs(r["bond_v"] - ref["bond_v"]))),
                          "rel_energy_gap_vs_two_row": abs(energy(r) - energy(ref)) / abs(energy(ref))}
    note("10x10 D=6 chi=72 ALS convergence")
    out["als"] = als_convergence(sess, st, cfg["chi"], ref)
    out["workload"] = "10x10 OBC PEPS, d=2, D=6, N(0,1) unit-norm sites, chi=72, 4 half-sweeps"
    return out


def cluster_windows(L, n):
    wins = []
    for i in range(L):
        for j in range(L):
            r0, r1 = max(0, i - (n + 1) // 2 + 1), min(L - 1, i + n // 2)
            c0, c1 = max(0, j - (n + 1) // 2 + 1), min(L - 1, j + n // 2)
            wins.append((0, r0, r1, c0, c1, i, j))
    return wins


def side_clusters(sess, binding, torch):
    """16x16, D=6, near-product, chi=36: all 256 n x n windows per call, FP32
    contractions (FP64 QR, norms and CU_0 boundaries), against the same
    windows in FP64."""
    from paper_1311_6696_amd.inputs import WORKLOADS, workload_peps
    cfg = WORKLOADS["16x16_D6_clusters"]
    L = cfg["L"]
    st = binding.to_device(workload_peps("16x16_D6_clusters"))
    out = {}
    for n in cfg["ns"]:
        wins = cluster_windows(L, n)

        def run(dtype, columns=False):
            envs = sess.cluster_env([st], wins, cfg["chi"], dtype, 4, columns=columns)
            res = sess.expect(envs)
            for e in envs:
                e.free()
            return res
        row = {"windows": len(wins)}
        res = {}
        for dt in ("f64", "f32"):
            note(f"16x16 D=6 clusters n={n} {dt}")
            run(dt)
            res[dt], t = timed(torch, lambda: run(dt), 1)
            fl = sum(r["flops"] for r in res[dt])
            row[dt] = {"windows_per_s": len(wins) / t, "s_per_call": t, "tflops": fl / t / 1e12,
                       "pct_peak": 100.0 * fl / t / 1e12 / PEAK[dt], "tflop_per_call": fl / 1e12}
        errs = [abs(a[k] - b[k]) for a, b in zip(res["f32"], res["f64"]) for k in ("sz", "right", "down")
                if not np.isnan(b[k])]
        e32 = sum(np.nansum([r["right"], r["down"]]) for r in res["f32"])
        e64 = sum(np.nansum([r["right"], r["down"]]) for r in res["f64"])
        row["f32"]["max_abs_err_vs_f64"] = float(max(errs))
        row["f32"]["rel_energy_err_vs_f64"] = abs(e32 - e64) / abs(e64)
        row["f32"]["speedup_vs_f64"] = row["f64"]["s_per_call"] / row["f32"]["s_per_call"]
        # the same windows with the bond downwards from the transposed window
        note(f"16x16 D=6 clusters n={n} f32 with column boundaries")
        run("f32", True)
        rc, tc = timed(torch, lambda: run("f32", True), 1)
        row["f32_columns"] = {"s_per_call": tc, "speedup_vs_f32": row["f32"]["s_per_call"] / tc,
                              "tflop_per_call": sum(r["flops"] for r in rc) / 1e12,
                              "max_down_gap_vs_two_row": float(np.nanmax([abs(a["down"] - b["down"])
                                                                          for a, b in zip(res["f32"], rc)]))}
        out[f"n{n}"] = row
    out["workload"] = ("16x16 OBC PEPS, d=2, D=6, near-product, chi=36, all 256 windows per n in one call, "
                       "FP32 contractions against FP64")
    return out


def side_instances(sess, binding, torch):
    """Independent lattices of mixed L and D in one call, chi = D^2: the D <= 5
    instances of the 32-instance draw and its smallest D = 8 one (L = 6).  The
    other eleven D = 8 instances (L = 8..12, hundreds of TFLOP each in FP64)
    exceed this measurement's time budget."""
    from paper_1311_6696_amd.inputs import batched_instances
    pairs, insts = batched_instances()
    d8 = sorted([k for k, (L, D) in enumerate(pairs) if D == 8], key=lambda k: pairs[k][0])[:1]
    keep = [k for k, (L, D) in enumerate(pairs) if D <= 5] + d8
    out = {}
    states = [binding.state_of(binding.to_device(insts[k])) for k in keep]
    chis = [pairs[k][1] ** 2 for k in keep]
    ref = None
    for dt in ("f64", "f32", "bf16"):
        note(f"batched instances {dt}")

        def run():
            # one call, one options record (chi = D^2) per lattice
            envs = sess.env_boundary(states, chis, dt, 4)
            res = sess.expect(envs)
            for e in envs:
                e.free()
            return res
        run()
        res, t = timed(torch, run, 1)
        fl = sum(r["flops"] for r in res)
        out[dt] = {"instances": len(keep), "instances_per_s": len(keep) / t, "s_per_batch": t,
                   "tflops": fl / t / 1e12, "pct_peak": 100.0 * fl / t / 1e12 / PEAK[dt], "tflop_per_batch": fl / 1e12}
        if dt == "f64":
            ref = res
        else:
            errs = [abs(energy(a) - energy(b)) / abs(energy(b)) for a, b in zip(res, ref)]
            out[dt]["max_rel_energy_err_vs_f64"] = float(max(errs))
            out[dt]["rel_energy_err_vs_f64_D8"] = float(errs[-1])
            out[dt]["speedup_vs_f64"] = out["f64"]["s_per_batch"] / t
    out["instances"] = [list(pairs[k]) for k in keep]
    out["workload"] = ("of 32 seeded lattices (L in 6..12, D in {3,4,5,8}, chi=D^2, U[0,1) entries): the "
                       f"{len(keep) - len(d8)} with D<=5 and the L=6 D=8 one, {len(keep)} lattices in one call")
    return out


def side_convergence(sess, binding, torch):
    """Convergence on synthetic states (the analogue of the paper's boundary
    and cluster studies, Secs. 5.2 and 5.3): 8x8, D=4, near-product and N(0,1)
    unit-norm sites.  Energy error of the full environment against chi (two-
    row and column sandwiches) with the boundary infidelity 1 - f of every
    row's boundaries, and of n x n cluster windows against n, all relative
    to the full environment at chi = 128."""
    from paper_1311_6696_amd.inputs import make_peps
    L, D = 8, 4
    out = {}
    for dist, seed in (("near_product", 1002), ("normal_unit", 1003)):
        st = binding.to_device(make_peps(L, L, D, dist, seed))
        note(f"convergence {dist}: reference chi=128")
        ref_env = sess.env_boundary([st], 128, "f64", 4)[0]
        ref = sess.expect([ref_env])[0]
        e_ref = energy(ref)
        rows = {}
        for chi in (4, 8, 16, 32, 64):
            for cols in (False, True):
                envs = sess.env_boundary([st], chi, "f64", 4, columns=cols)
                r = sess.expect(envs)[0]
                fid = {}
                if not cols:
                    # boundary fidelity against the chi = 128 boundaries, every row from both sides
                    ov = sess.ctx.boundary_overlap([(envs[0], ref_env, s, k) for s in (0, 1) for k in range(1, L)])
                    inf = [1.0 - abs(xy) / np.sqrt(xx * yy) for xy, xx, yy in ov]
                    fid = {"max_boundary_infidelity": float(max(inf)), "mean_boundary_infidelity": float(np.mean(inf))}
                for e in envs:
                    e.free()
                rows[f"chi{chi}" + ("_columns" if cols else "")] = {**fid,
                    "rel_energy_err": abs(energy(r) - e_ref) / abs(e_ref),
                    "max_bond_err": float(max(np.max(np.abs(r["bond_h"] - ref["bond_h"])),
                                              np.max(np.abs(r["bond_v"] - ref["bond_v"])))),
                    "log_norm_err": abs(r["log_norm"] - ref["log_norm"])}
        clusters = {}
        for n in (2, 3, 4, 6, 8):
            note(f"convergence {dist}: clusters n={n}")
            wins = []
            for i in range(L):
                for j in range(L):
                    r0, r1 = max(0, i - (n + 1) // 2 + 1), min(L - 1, i + n // 2)
                    c0, c1 = max(0, j - (n + 1) // 2 + 1), min(L - 1, j + n // 2)
                    wins.append((0, r0, r1, c0, c1, i, j))
            envs = sess.cluster_env([st], wins, 32, "f64", 4)
            res = sess.expect(envs)
            for e in envs:
                e.free()
            e_cl = float(sum(np.nansum([r["right"], r["down"]]) for r in res))
            clusters[f"n{n}"] = {"rel_energy_err": abs(e_cl - e_ref) / abs(e_ref)}
        ref_env.free()
        out[dist] = {"energy_ref": e_ref, "environment_vs_chi": rows, "clusters_chi32_vs_n": clusters}
    out["workload"] = ("8x8 OBC PEPS, d=2, D=4, near-product (seed 1002) and N(0,1) unit-norm (seed 1003) "
                       "sites, 4 ALS half-sweeps; reference: full environment at chi=128")
    return out


EVOLUTION = {"steps": 20, "taus": (0.1, 0.05, 0.02)}


def side_evolution(sess, binding, torch):
    """Imaginary-time full updates of the 4x4 Heisenberg model from a Neel
    start (the driver over the site and bond environments), D = 2, 3, 4 at
    lossless chi: energy per site against the exact -0.57432544 and time per
    Trotter step (four environments plus six bond fits per bond set)."""
    from paper_1311_6696_amd import evolve
    out = {}
    taus, n = EVOLUTION["taus"], EVOLUTION["steps"]
    for D, chi, steps in ((2, 16, n), (3, 81, n), (4, 256, n)):
        note(f"evolution 4x4 D={D}")
        A = evolve.neel_start(4, 4, D, 1e-1, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trace = []
        for k, tau in enumerate(taus):
            A, more = evolve.full_update(sess, A, tau, steps, chi, cutoff=1e-10, every=10)
            trace += [(k * steps + s, e) for s, e in more]
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[f"D{D}"] = {"chi": chi, "tau": list(taus), "steps": len(taus) * steps, "energy_per_site": [e for _, e in trace],
                        "best": min(e for _, e in trace), "exact": -0.57432544,
                        "ms_per_step_incl_energy_checks": 1000.0 * t / (len(taus) * steps)}
    out["workload"] = ("4x4 OBC Heisenberg, Neel start with 0.1 noise, exp(-tau S.S) gates (tau " + ", ".join(map(str, taus)) + "), "
                       "3 alternating fits per bond, bond rebalancing")
    return out


SIDE = {"precision": side_precision, "clusters": side_clusters, "instances": side_instances,
        "convergence": side_convergence, "evolution": side_evolution}
DEFAULT_WORKLOADS = ("precision", "clusters", "instances")


def cpu_info():
    """Host CPU model and the BLAS behind NumPy (name, threads)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas, threads = "unknown", os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        libs = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if libs:
            blas = f"{libs[0].get('internal_api')} {libs[0].get('version')}"
            threads = max(i.get("num_threads", 1) for i in libs)
    except Exception:
        pass
    return model, blas, threads


def chain2_io_bytes(L, D, chi, d=2):
    """Algorithmic bytes of one two-row column step (inputs and output once,
    FP64): the incoming and outgoing column environments (chi D^2 D^2 chi
    each), the top and bottom boundary tensors (chi D^2 chi each) and the
    two rows' site tensors (d D^4 each)."""
    return 8.0 * (2 * chi * D ** 4 * chi + 2 * chi * D * D * chi + 2 * d * D ** 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--halfsweeps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32/BF16 measurements")
    ap.add_argument("--no-site-env", action="store_true",
                    help="skip the measurement of the single-site norm environments")
    ap.add_argument("--no-columns", action="store_true",
                    help="skip the measurement of vertical bonds from column boundaries")
    ap.add_argument("--batch", type=int, default=8,
                    help="lattices per call of the batched side measurement (1 = skip)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the default side workloads: precision (10x10 D=6 chi=72 in FP64/FP32/BF16), "
                         "clusters (16x16 D=6 n x n windows, FP32 and FP64), instances (batched lattices, "
                         "FP64 and BF16)")
    ap.add_argument("--workloads", default="",
                    help="comma list of further side workloads: convergence (energy error against chi and "
                         "cluster size n), evolution (4x4 imaginary-time full updates)")
    ap.add_argument("--evolution-steps", type=int, default=20, help="Trotter steps per tau of the evolution workload")
    ap.add_argument("--evolution-taus", default="0.1,0.05,0.02", help="tau schedule of the evolution workload")
    ap.add_argument("--autotune", action="store_true",
                    help="time the contraction launch shapes on one untimed environment first")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the library's launch sequences from captured HIP graphs")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="one device-to-device copy of this many MiB before the run: a plain copy kernel of "
                         "known size against which hardware byte counters are scaled")
    args = ap.parse_args()
    EVOLUTION["steps"] = args.evolution_steps
    EVOLUTION["taus"] = tuple(float(x) for x in args.evolution_taus.split(","))
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path has no multi-GPU component); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_6696_amd import binding
    from paper_1311_6696_amd.inputs import WORKLOADS, workload_peps

    cfg = WORKLOADS["8x8_D4_chi32"]
    A = workload_peps("8x8_D4_chi32")
    chi, H = cfg["chi"], args.halfsweeps
    sess = binding.Session(0)
    if args.graphs:
        sess.ctx.graphs(True)
    # the lattice's device pointers marshalled once (the inputs stay resident)
    dev_state = binding.state_of(binding.to_device(A))
    torch.cuda.synchronize()
    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.autotune:
        note("autotuning launch shapes on one environment")
        sess.ctx.autotune(1)
        run_steps(sess, dev_state, chi, "f64", H, 1)
        sess.ctx.autotune(0)
    note("warm-up")
    # warm-up, then the timed region (bracketed by synchronisations)
    ref = run_steps(sess, dev_state, chi, "f64", H, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    split = []
    res = run_steps(sess, dev_state, chi, "f64", H, args.steps, split)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1000.0 * dt / args.steps
    flops = res["flops"]

    note(f"timed {args.steps} steps: {ms:.2f} ms/step")
    # contraction-kernel statistics: HIP events around every launch on the library's stream
    sess.ctx.profile(True)
    run_steps(sess, dev_state, chi, "f64", H, max(2, args.steps // 4))
    torch.cuda.synchronize()
    fl, kms, nl, nbytes = sess.ctx.stats()
    sess.ctx.profile(False)
    # The dominant kernel is the variant that carries most of the step's
    # algorithmic flops.  (Event-bracketed totals overstate variants with many
    # short launches: each bracket adds a few microseconds.)  Its launches are
    # long, so the event-timed average matches the profiler's duration.
    dom = int(np.argmax(fl))
    nlaunch = max(int(nl[dom]), 1)
    per_launch_flops = fl[dom] / nlaunch
    per_launch_bytes = nbytes[dom] / nlaunch
    avg_ms = kms[dom] / nlaunch
    kernel = binding.variant_name(dom)
    # The path is a chain of dense contractions whose algorithmic traffic is
    # only each step's inputs and outputs: the roofline is the FP64 MFMA peak.
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    tc_total_ms = float(np.sum(kms)) / max(2, args.steps // 4)
    traffic = measured_traffic(kernel)
    # Launches are set against the I/O of the two-row column steps they carry,
    # counted in full-bond (chi) steps through the flops of one such step:
    # the fused two-row kernel does, per (x, e) pair of bonds, the incoming
    # environment times the top boundary (D^6 chi MACs), the four layers
    # (d D^8 each) and the bottom boundary (D^6 chi); the fused ket-bra
    # kernel applies the two layers of one row, 8 d D^8 chi^2 flops per step.
    D, d = cfg["D"], 2
    if kernel.startswith("k2_kernel"):
        step_flops = 2.0 * chi * chi * (2 * D ** 6 * chi + 4 * d * D ** 8)
    else:
        step_flops = 8.0 * d * D ** 8 * chi * chi
    steps_per_launch = per_launch_flops / step_flops
    chain_io = steps_per_launch * chain2_io_bytes(cfg["L"], D, chi, d)

    out = {
        "metric": "env contractions/sec + GFLOP/s (% MFMA peak), FP64 vs BF16/FP32 at stated err",
        "value": args.steps / dt,
        "unit": "env/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded near-product PEPS, no optimised states available)",
        "config": {"workload": "full environment of an 8x8 OBC PEPS, d=2, D=4, near-product, chi=32, "
                               f"{H} ALS half-sweeps per truncated row; norm, 64 <Sz>, 112 bond energies",
                   "lattice": "8x8", "D": 4, "chi": chi, "halfsweeps": H, "parallelism": "single GPU"},
        "graph_replay": bool(args.graphs),
        "autotuned": bool(args.autotune),
        "gflops_per_s": flops / (ms * 1e-3) / 1e9,
        "pct_fp64_mfma_peak": 100.0 * flops / (ms * 1e-3) / (PEAK["f64"] * 1e12),
        "gflop_per_env": flops / 1e9,
        "boundary_ms": 1000.0 * float(np.median([s[0] for s in split])),
        "expect_ms": 1000.0 * float(np.median([s[1] for s in split])),
        "roofline": {
            "bound": "mfma",
            "kernel": kernel,
            "achieved": achieved,
            "peak": PEAK["f64"],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK["f64"],
            "traffic": traffic,
            "flops_per_launch": per_launch_flops,
            "operand_bytes_per_launch": per_launch_bytes,
            "chain_io_bytes_per_launch": chain_io,
            "traffic_over_chain_io": (traffic / chain_io) if traffic else None,
            "launches_per_env": int(nl[dom] / max(2, args.steps // 4)),
            "avg_launch_us": 1000.0 * avg_ms,
            "contraction_ms_per_env": tc_total_ms,
        },
    }
    note("ALS convergence")
    out["als"] = als_convergence(sess, dev_state, chi, res, H)

    if args.batch > 1:
        # the same workload, several independent lattices per call (one grouped launch per stage)
        note(f"batched: {args.batch} and {4 * args.batch} lattices per call")
        states = [binding.state_of(binding.to_device(workload_peps("8x8_D4_chi32", seed=2000 + i)))
                  for i in range(4 * args.batch)]

        def batched(dtype, nlat):
            sub = states[:nlat]
            for _ in range(2):
                envs = sess.env_boundary(sub, chi, dtype, H)
                sess.expect(envs)
                for e in envs:
                    e.free()
            torch.cuda.synchronize()
            nb = max(2, args.steps // 4)
            t0 = time.perf_counter()
            for _ in range(nb):
                envs = sess.env_boundary(sub, chi, dtype, H)
                res = sess.expect(envs)
                for e in envs:
                    e.free()
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            return nb * nlat / tb, 1000.0 * tb / nb, res

        single = args.steps / dt
        v, ms, _ = batched("f64", args.batch)
        out["batched"] = {"lattices_per_call": args.batch, "value": v, "unit": "env/s", "ms_per_call": ms,
                          "speedup_vs_single_f64": v / single}
        # the batched forms (4x the lattices per call) against the plain
        # single-lattice FP64 rate, each lattice's energy against its own FP64 result
        nl = 4 * args.batch
        v64, ms64, r64 = batched("f64", nl)
        e64 = [energy(r) for r in r64]
        forms = {"lattices_per_call": nl, "single_f64_env_per_s": single}
        for dname in ("f64", "f32"):
            vv, mm, rr = (v64, ms64, r64) if dname == "f64" else batched(dname, nl)
            err = max(abs(energy(r) - e) / abs(e) for r, e in zip(rr, e64))
            forms[dname] = {"value": vv, "unit": "env/s", "ms_per_call": mm, "speedup_vs_single_f64": vv / single,
                            "max_rel_energy_err_vs_f64": err}
        # the dominant kernel of the batched FP64 call (same rule as the headline's roofline)
        sess.ctx.profile(True)
        envs = sess.env_boundary(states[:nl], chi, "f64", H)
        sess.expect(envs)
        for e in envs:
            e.free()
        torch.cuda.synchronize()
        bfl, bkms, bnl, _ = sess.ctx.stats()
        sess.ctx.profile(False)
        bd = int(np.argmax(bfl))
        if bnl[bd] > 0 and bkms[bd] > 0:
            rate = bfl[bd] / (bkms[bd] * 1e-3) / 1e12
            forms["f64"]["dominant_kernel"] = {"kernel": binding.variant_name(bd), "achieved": rate,
                                               "peak": PEAK["f64"], "unit": "TFLOP/s", "frac": rate / PEAK["f64"],
                                               "launches": int(bnl[bd]),
                                               "avg_launch_us": 1000.0 * bkms[bd] / bnl[bd]}
        out["batched_forms"] = forms

    if not args.no_columns:
        # the same workload with the vertical bonds from single-column sandwiches of
        # the left/right boundaries (built in the same batched run as the row ones)
        note("vertical bonds from column boundaries")
        run_steps(sess, dev_state, chi, "f64", H, 2, columns=True)
        torch.cuda.synchronize()
        n = max(3, args.steps // 2)
        csplit = []
        t0 = time.perf_counter()
        rc = run_steps(sess, dev_state, chi, "f64", H, n, csplit, columns=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out["columns"] = {"value": n / t, "unit": "env/s", "ms_per_step": 1000.0 * t / n,
                          "speedup_vs_two_row": (n / t) / (args.steps / dt), "gflop_per_env": rc["flops"] / 1e9,
                          "boundary_ms": 1000.0 * float(np.median([s[0] for s in csplit])),
                          "expect_ms": 1000.0 * float(np.median([s[1] for s in csplit])),
                          "max_bond_v_gap_vs_two_row": float(np.max(np.abs(rc["bond_v"] - res["bond_v"]))),
                          "max_bond_h_diff": float(np.max(np.abs(rc["bond_h"] - res["bond_h"])))}

    if not args.no_site_env:
        # norm environments N_l of all 64 sites of one environment, one batched call
        note("site norm environments")
        env = sess.env_boundary([dev_state], chi, "f64", H)[0]
        sites = [(env, r, c) for r in range(len(A)) for c in range(len(A[0]))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sess.site_env(sites)   # forms and keeps the row sandwiches
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        n = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(n):
            got, sfl = sess.site_env(sites)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n
        env.free()
        out["site_env"] = {"sites_per_call": len(sites), "ms_per_call": 1000.0 * t, "value": len(sites) / t,
                           "unit": "site environments/s", "gflop_per_call": sfl / 1e9,
                           "tflops": sfl / t / 1e12, "first_call_ms": 1000.0 * t_first,
                           "row_sandwiches": "formed by the first call and kept with the environment; "
                                             "ms_per_call is the mean of the later calls"}
        # right-hand sides b of both sites of all 56 horizontal bonds under one
        # imaginary-time Heisenberg gate exp(-0.02 S.S), one batched call
        note("gated bond environments")
        h = np.zeros((4, 4))
        sz, sp = np.diag([0.5, -0.5]), np.array([[0.0, 1.0], [0.0, 0.0]])
        h += np.kron(sz, sz) + 0.5 * (np.kron(sp, sp.T) + np.kron(sp.T, sp))
        ev, U = np.linalg.eigh(h)
        gate = torch.as_tensor((U @ np.diag(np.exp(-0.02 * ev)) @ U.T).reshape(2, 2, 2, 2), device="cuda")
        env = sess.env_boundary([dev_state], chi, "f64", H)[0]
        bonds = [(env, r, c, gate) for r in range(len(A)) for c in range(len(A[0]) - 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sess.bond_env(bonds)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(n):
            got, bfl = sess.bond_env(bonds)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / n
        env.free()
        out["bond_env"] = {"bonds_per_call": len(bonds), "ms_per_call": 1000.0 * t, "value": len(bonds) / t,
                           "unit": "gated bond environments/s", "gflop_per_call": bfl / 1e9,
                           "tflops": bfl / t / 1e12, "first_call_ms": 1000.0 * t_first,
                           "row_sandwiches": "formed by the first call and kept with the environment; "
                                             "ms_per_call is the mean of the later calls"}

    if not args.no_forms:
        forms = {}
        e64 = energy(res)
        for dt_name in ("f32", "bf16"):
            note(f"precision form {dt_name}")
            r = run_steps(sess, dev_state, chi, dt_name, H, 2)
            torch.cuda.synchronize()
            n = max(3, args.steps // 2)
            t0 = time.perf_counter()
            r = run_steps(sess, dev_state, chi, dt_name, H, n)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            forms[dt_name] = {"value": n / t, "unit": "env/s", "speedup_vs_f64": (n / t) / (args.steps / dt),
                              "rel_energy_err_vs_f64": abs(energy(r) - e64) / abs(e64),
                              "max_bond_err_vs_f64": float(max(np.max(np.abs(r["bond_h"] - res["bond_h"])),
                                                               np.max(np.abs(r["bond_v"] - res["bond_v"]))))}
        out["precision_forms"] = forms

    side = [] if args.no_workloads else list(DEFAULT_WORKLOADS)
    side += [w for w in args.workloads.split(",") if w and w not in side]
    if side:
        out["workloads"] = {}
    for w in side:
        out["workloads"][w] = SIDE[w](sess, binding, torch)

    if not args.no_cpu:
        # the oracle as it stands, on the host cores, on the same workload: the
        # boundaries (median of three runs) plus the sandwiches (one run)
        note("oracle cpu baseline")
        from oracle import api
        model, blas, threads = cpu_info()
        tb = []
        for _ in range(3):
            t0 = time.perf_counter()
            oenv = api.env_boundary(A, chi, H)
            tb.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        r_cpu = api.expect(oenv)
        te = time.perf_counter() - t0
        t = float(np.median(tb)) + te
        out["cpu_baseline"] = {"value": 1.0 / t, "unit": "env/s", "cores": threads, "kind": "oracle",
                               "sample": "the same 8x8 D=4 chi=32 environment: top and bottom boundaries "
                                         f"(median of 3 runs, {np.median(tb):.1f} s) plus the one- and two-row "
                                         f"sandwiches (one run, {te:.1f} s); NumPy FP64",
                               "cpu_model": model, "blas": blas,
                               "boundary_s_runs": tb, "sandwich_s": te}
        out["max_abs_diff_vs_oracle"] = float(max(np.max(np.abs(res[k] - r_cpu[k]))
                                                  for k in ("sz", "bond_h", "bond_v")))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
