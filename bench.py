"""Benchmark of the mixed-precision Jacobi eigensolver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full eigendecomposition through the hot path (jacobi_eigh_mixed:
FP32 Jacobi -> FP64 Newton-Schulz -> Q_d^T A Q_d -> FP64 Jacobi -> sorted
output) of one seeded synthetic matrix already resident in HBM.  The plain
FP64 Jacobi (jacobi_eigh) is timed on the same matrix for comparison.  One
JSON line is printed; see the field descriptions in main().
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "eigendecomps/sec, mixed vs plain FP64 Jacobi on MI355X at residual ≤1e-13·n"
PEAK = {"f64": 78.6, "f32": 157.3}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                      # GB/s

WORKLOADS = {
    "goe4096": dict(n=4096, desc="A=(G+G^T)/2, G iid N(0,1), seed 3"),
    "geo1024": dict(n=1024, desc="A=Q diag(lam) Q^T, lam_i=+-10^(-6i/(n-1)), Haar Q, seed 2"),
    "geo4096": dict(n=4096, desc="A=Q diag(lam) Q^T, |lam_i|=100^(-i/(n-1)), random signs, "
                                 "Haar Q, seed 8"),
    "ari4096": dict(n=4096, desc="A=Q diag(lam) Q^T, |lam_i|=1-(i/(n-1))(1-1/100), random "
                                 "signs, Haar Q, seed 6"),
    "blk4096": dict(n=4096, desc="8 decoupled diagonal blocks of 512, A_i=Q_i diag(lam_i) "
                                 "Q_i^T, lam_i ~ U[-1,1], Haar Q_i, seed 9"),
}


def make_input(name):
    import workloads as wl
    if name == "goe4096":
        return wl.goe(4096, 3), None
    if name == "geo1024":
        A, lam = wl.geo_spectrum(1024, 2)
        return A, lam
    if name == "geo4096":
        return wl.geo_spectrum(4096, 8, kappa=1e2)
    if name == "ari4096":
        return wl.ari_spectrum(4096, 6, kappa=1e2)
    if name == "blk4096":
        return wl.block_diagonal(4096, 8, 9)
    raise SystemExit(f"unknown workload {name}")


def _tiles(n, b):
    N = -(-n // b)
    N += N % 2
    npairs = N // 2
    M = 2 * b
    nbt = npairs * (npairs - 1) // 2      # off-diagonal pair tiles k < l of B
    nvt = (N * b // M) * npairs           # row tiles x pairs of V
    return M, nbt, nvt


def apply_flops(n, b, part):
    """Algorithmic flops of one update launch (one round).  part "B": every
    off-diagonal pair tile k < l becomes U_k^T B_kl U_l, two (2b)^3 products
    (the mirror tile is its transpose, not recomputed); part "V": every row
    tile of V becomes V U_l, one (2b)^3 product."""
    M, nbt, nvt = _tiles(n, b)
    return 2.0 * M ** 3 * (2 * nbt if part == "B" else nvt)


def apply_bytes(n, b, elem, part):
    """Algorithmic HBM bytes of one update launch: each off-diagonal pair tile
    of B read and written once (B keeps only its upper b x b blocks during the
    sweeps, so a tile is four stored blocks in either orientation); V tiles
    read and written once.  The small U blocks are cache resident and not
    counted."""
    M, nbt, nvt = _tiles(n, b)
    tile = M * M * elem
    return tile * (2 * nbt if part == "B" else 2 * nvt)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "update_kernels_goe4096_traffic.md")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary (already scaled by the copy-probe factors), or
    None when there is none for this workload or a kernel source has changed
    since the counters were taken (the summary records the source hashes)."""
    import hashlib
    import re
    if workload != "goe4096" or not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    for path, h in re.findall(r"- `([^`]+)`: `([0-9a-f]+)`", text):
        full = os.path.join(ROOT, path)
        if not os.path.exists(full) or \
                hashlib.sha256(open(full, "rb").read()).hexdigest()[:len(h)] != h:
            return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == kernel:
            return int(float(cells[4]))
    return None


def oracle_sweeps_estimate(name, n):
    """The oracle's sweep count for this workload: read from the fixture when
    the oracle was run at this size, else extrapolated linearly in log2(n) from
    the oracle's sweep counts on the same distribution at smaller n."""
    gold = os.path.join(ROOT, "tests", "golden")
    if name == "geo1024":
        with open(os.path.join(gold, "oracle_geo1024.txt")) as f:
            for line in f:
                if line.startswith("# n "):
                    return float(line.split()[4]), "oracle run (tests/golden/oracle_geo1024.txt)"
    path = os.path.join(gold, "oracle_goe_sweeps.txt")
    pts = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            nn, sw = line.split()[:2]
            pts.append((math.log2(float(nn)), float(sw)))
    x = np.array([p[0] for p in pts])
    y = np.array([p[1] for p in pts])
    slope, icpt = np.polyfit(x, y, 1)
    est = slope * math.log2(n) + icpt
    return float(est), ("log2(n) fit of oracle sweep counts at n=" +
                        ",".join(str(int(2 ** v)) for v in x))


def cpu_baseline(name, A, budget_s=12.0):
    """Time the CPU oracle on a bounded sample of the same workload: pivot rows
    of the first cyclic-by-row sweep on this very matrix, until budget_s of
    CPU time, then scale by the oracle's sweeps per eigendecomposition."""
    import oracle
    n = A.shape[0]
    B = np.array(A, dtype=np.float64, copy=True)
    V = np.eye(n)
    rows, rot = 0, 0
    t0 = time.process_time()
    w0 = time.perf_counter()
    while time.process_time() - t0 < budget_s and rows < n - 1:
        step = 4 if n > 2048 else 32
        rot += oracle.jacobi_rows(B, V, rows, rows + step)
        rows += step
    cpu_s = time.process_time() - t0
    wall = time.perf_counter() - w0
    rate = rot / wall
    sweeps, how = oracle_sweeps_estimate(name, n)
    per_eig = sweeps * n * (n - 1) / 2.0
    return {
        "value": rate / per_eig,
        "unit": "eigendecomps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{rows} pivot rows ({rot} rotations, {wall:.1f} s wall, {cpu_s:.1f} s CPU) "
                   f"of the first cyclic-by-row sweep on the same n={n} matrix; "
                   f"{rate:.0f} rotations/s scaled by {sweeps:.1f} sweeps x n(n-1)/2 "
                   f"rotations per eigendecomposition ({how})"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="goe4096", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 256 MiB device-to-device copy three times (the "
                         "reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver is a "
              "single-GPU library", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_00495_amd as pj
    if not os.path.exists(pj.LIB_PATH):
        raise SystemExit("libjacobi.so is not built: run python -c 'import __graft_entry__ as g; g.build()'")
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.copy_probe:
        x = torch.ones(1 << 25, dtype=torch.float64, device="cuda")  # 256 MiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8, "launches": 3}), flush=True)
        return

    wl_name = args.workload
    A, lam = make_input(wl_name)
    n = A.shape[0]
    At = torch.tensor(A, device="cuda")
    opts = pj.make_opts()
    topts = pj.make_opts(timing=1)  # per-kernel HIP events: separate, untimed pass
    ws = pj.Workspace()

    def run_mixed(o=opts):
        return pj.eigh_mixed(At, opts=o, ws=ws, return_info=True)

    def run_plain():
        return pj.eigh(At, opts=opts, ws=ws, return_info=True)

    for _ in range(args.warmup):
        run_mixed()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        W, V, info = run_mixed()
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    plain = None
    if not args.no_plain:
        for _ in range(args.warmup):
            run_plain()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pinfos = []
        for _ in range(args.steps):
            Wp, Vp, pinfo = run_plain()
            pinfos.append(pinfo)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t1
        plain = {"value": args.steps / dtp, "ms_per_step": 1e3 * dtp / args.steps,
                 "sweeps": pinfos[-1]["sweeps"], "orth_est": pinfos[-1]["orth_est"],
                 "orth_refresh": pinfos[-1]["polished"],
                 "skipped_tiles": pinfos[-1]["skipped_tiles"]}

    # accuracy of the timed output (properties that hold at any size)
    Wn, Vn = W.cpu().numpy(), V.cpu().numpy()
    nrmF = np.linalg.norm(A)
    acc = {
        "residual_rel_F": float(np.linalg.norm(A @ Vn - Vn * Wn) / nrmF),
        "residual_bar": 1e-13 * n,
        "orth_F": float(np.linalg.norm(Vn.T @ Vn - np.eye(n))),
        "orth_bar": 1e-14 * n,
        "trace_rel_err": float(abs(Wn.sum() - np.trace(A)) / np.abs(A).sum()),
        "frobenius_rel_err": float(abs(math.sqrt((Wn ** 2).sum()) - nrmF) / nrmF),
    }
    if lam is not None:
        acc["eig_err_vs_known_spectrum"] = float(np.abs(Wn - lam).max() / np.abs(lam).max())
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{wl_name}.txt")
    if os.path.exists(gold):
        Wo = np.loadtxt(gold, ndmin=2)[:, 0]
        acc["eig_err_vs_oracle"] = float(np.abs(Wn - Wo).max() / np.abs(Wo).max())
        if lam is not None:
            acc["oracle_err_vs_known_spectrum"] = float(np.abs(Wo - lam).max() / np.abs(lam).max())
        acc["eig_bar"] = 1e-13
    if plain is not None:
        acc["mixed_vs_plain_max_dW_rel"] = float(
            np.abs(Wn - Wp.cpu().numpy()).max() / np.abs(Wn).max())
    gate = acc["residual_rel_F"] <= acc["residual_bar"] and acc["orth_F"] <= acc["orth_bar"]
    if "eig_err_vs_known_spectrum" in acc:
        # the exact spectrum decides; the oracle's stored eigenvalues (the
        # diagonal after its sweeps) are themselves ~2.5e-13 off at n = 1024
        gate = gate and acc["eig_err_vs_known_spectrum"] <= 1e-13
    elif "eig_err_vs_oracle" in acc:
        gate = gate and acc["eig_err_vs_oracle"] <= 1e-13
    acc["gate_passed"] = bool(gate)

    # roofline of the dominant update kernel, from the in-library HIP events of
    # one instrumented (untimed) solve: events around every launch on its stream
    infos = [run_mixed(topts)[2]]
    torch.cuda.synchronize()
    last = infos[-1]
    b = last["block"]

    def tot(key, idx):
        return sum(i[key][idx] for i in infos)

    cands = {
        "apply_B_f32": (tot("t_apply_ms", 1), tot("n_apply", 1), "B", "f32"),
        "apply_V_f32": (tot("t_applyv_ms", 1), tot("n_applyv", 1), "V", "f32"),
        "apply_B_f64": (tot("t_apply_ms", 0), tot("n_apply", 0), "B", "f64"),
        "apply_V_f64": (tot("t_applyv_ms", 0), tot("n_applyv", 0), "V", "f64"),
    }
    kern_ms = {k: round(v[0], 2) for k, v in cands.items()}
    kern_ms["pair_solve_f32"] = round(tot("t_pair_ms", 1), 2)
    kern_ms["pair_solve_f64"] = round(tot("t_pair_ms", 0), 2)
    # the FP32 V update runs inside the pair-solve launch in the timed solves
    # (the instrumented solve times it as its own kernel), so the dominant
    # kernel is taken among the update kernels the timed solves launch as such
    dom = max((k for k in cands if k != "apply_V_f32"), key=lambda k: cands[k][0])
    t_ms, cnt, part, dtype = cands[dom]
    avg_s = t_ms / max(cnt, 1) / 1e3
    elem = 4 if dtype == "f32" else 8
    flops = apply_flops(n, b, part)
    nbytes = apply_bytes(n, b, elem, part)
    # the bound is whichever floor is higher for this launch's algorithmic work
    mfma_bound = flops / (PEAK[dtype] * 1e12) >= nbytes / (HBM_PEAK * 1e9)
    names = {("B", "f32"): "update_b_kernel<float, 64>",
             ("V", "f32"): "update_v_kernel<float, 64>",
             ("B", "f64"): "update_b_kernel<double, 64>",
             ("V", "f64"): "update_v_kernel<double, 64>"}
    achieved = flops / avg_s / 1e12 if mfma_bound else nbytes / avg_s / 1e9
    peak = PEAK[dtype] if mfma_bound else HBM_PEAK
    roofline = {
        "kernel": "lj::" + names[(part, dtype)] + (" (off-diagonal B tiles)" if part == "B"
                                                   else " (V row tiles)"),
        "bound": "mfma" if mfma_bound else "hbm",
        "achieved": round(achieved, 2),
        "peak": peak,
        "unit": "TFLOP/s" if mfma_bound else "GB/s",
        "frac": round(achieved / peak, 4),
        "traffic": measured_traffic(names[(part, dtype)], wl_name),
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-probe scaled)",
        "avg_launch_us": round(avg_s * 1e6, 2),
        "launches": cnt,
        "flops_per_launch": flops,
        "bytes_per_launch": nbytes,
        "achieved_TFLOPs": round(flops / avg_s / 1e12, 2),
        "achieved_GBps": round(nbytes / avg_s / 1e9, 1),
        "kernel_ms_per_step": kern_ms,
    }

    cpu = None
    # the oracle's sweep count is known (fixture) or fitted (GOE runs) only
    # for these two workloads; the others report no CPU baseline
    if not args.no_cpu_baseline and wl_name in ("goe4096", "geo1024"):
        cpu = cpu_baseline(wl_name, A)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "eigendecomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": wl_name,
            "n": n,
            "input": WORKLOADS[wl_name]["desc"],
            "path": "jacobi_eigh_mixed",
            "block": b,
            "sweeps32": last["sweeps32"],
            "sweeps64": last["sweeps"],
            "ns_iters": last["ns_iters"],
            "orth_est": last["orth_est"],
            "orth_refresh": last["polished"],
            "skipped_tiles": last["skipped_tiles"],
        },
        "plain_fp64": plain,
        "speedup_vs_plain": None if plain is None else round(value / plain["value"], 3),
        "accuracy": acc,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
