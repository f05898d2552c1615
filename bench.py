"""Throughput of full boundary-MPS environments on one MI355X.

One step = one complete environment of the 8x8, D=4, chi=32 near-product
PEPS (top and bottom boundaries by ALS row absorption, then the norm, 64
<S^z> and 112 Heisenberg bond energies from the one- and two-row
sandwiches), inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
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
def run_steps(sess, dev_state, chi, dtype, halfsweeps, n, split=None):
    """n full environments; `split` (a list) receives (boundary_s, expect_s) per step."""
    res = None
    for _ in range(n):
        t0 = time.perf_counter()
        envs = sess.env_boundary([dev_state], chi, dtype, halfsweeps)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--halfsweeps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32/BF16 measurements")
    ap.add_argument("--batch", type=int, default=8,
                    help="lattices per call of the batched side measurement (1 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path has no multi-GPU component); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_6696_amd import binding
    from paper_1311_6696_amd.inputs import CONFIGS, config_peps

    cfg = CONFIGS[2]
    A = config_peps(2)
    chi, H = cfg["chi"], args.halfsweeps
    sess = binding.Session(0)
    dev_state = binding.to_device(A)
    torch.cuda.synchronize()

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
    fl, kms, nl = sess.ctx.stats()
    sess.ctx.profile(False)
    dom = int(np.argmax(kms))
    per_launch_flops = fl[dom] / max(nl[dom], 1)
    avg_ms = kms[dom] / max(nl[dom], 1)
    achieved = per_launch_flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    tc_total_ms = float(np.sum(kms)) / max(2, args.steps // 4)

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
        "gflops_per_s": flops / (ms * 1e-3) / 1e9,
        "pct_fp64_mfma_peak": 100.0 * flops / (ms * 1e-3) / (PEAK["f64"] * 1e12),
        "gflop_per_env": flops / 1e9,
        "boundary_ms": 1000.0 * float(np.median([s[0] for s in split])),
        "expect_ms": 1000.0 * float(np.median([s[1] for s in split])),
        "roofline": {
            "bound": "mfma",
            "kernel": binding.variant_name(dom),
            "achieved": achieved,
            "peak": PEAK["f64"],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK["f64"],
            "traffic": None,
            "launches_per_env": int(nl[dom] / max(2, args.steps // 4)),
            "avg_launch_us": 1000.0 * avg_ms,
            "contraction_ms_per_env": tc_total_ms,
        },
    }

    if args.batch > 1:
        # the same workload, several independent lattices per call (one grouped launch per stage)
        note(f"batched: {args.batch} lattices per call")
        states = [binding.to_device(config_peps(2, seed=2000 + i)) for i in range(args.batch)]
        for _ in range(2):
            envs = sess.env_boundary(states, chi, "f64", H)
            sess.expect(envs)
        torch.cuda.synchronize()
        nb = max(2, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(nb):
            envs = sess.env_boundary(states, chi, "f64", H)
            sess.expect(envs)
            for e in envs:
                e.free()
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        out["batched"] = {"lattices_per_call": args.batch, "value": nb * args.batch / tb, "unit": "env/s",
                          "ms_per_call": 1000.0 * tb / nb}

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

    if not args.no_cpu:
        note("oracle cpu baseline")
        # the oracle as it stands, on the host cores, on one full environment of the same workload
        from oracle import api
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = os.cpu_count()
        t0 = time.perf_counter()
        r_cpu = api.expect(api.env_boundary(A, chi, H))
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / t, "unit": "env/s", "cores": cores, "kind": "oracle",
                               "sample": "one full environment of the same 8x8 D=4 chi=32 workload "
                                         f"({t:.1f} s, NumPy/OpenBLAS FP64)"}
        out["max_abs_diff_vs_oracle"] = float(max(np.max(np.abs(res[k] - r_cpu[k]))
                                                  for k in ("sz", "bond_h", "bond_v")))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
