"""Benchmark of the TT-contraction hot path on one MI355X.

One step = one pass over every operation of the path, each at its full
workload size, inputs resident in HBM:
  pair10 : order-10 FP32 pair (modes 16, ranks 32): inner product, contraction
           over modes 1-5 written as the natural-order TT (ranks 32*32),
           mode-n product of all ten modes with 16x16 matrices, and the
           gradient of the inner product with respect to every core;
  mpo8   : order-8 MPO (I = J = 32, rank 16) x order-8 TT (mode 32, rank 64),
           BF16 inputs, FP32 output with ranks 1024;
  batch  : 4096 uneven FP32 pairs, inner product + junction of the last two
           positions each, one persistent launch (graph replay);
  layer4 : order-4 TT-matrix 4096 -> 4096 (modes 8, ranks 32) on a
           8192 x 4096 FP32 batch: forward, MSE loss, backward (dX and every
           core gradient).
value = TT contractions per step / seconds per step.  Beside the step, the
BF16 batch, the per-pair launch loop and the BF16-MFMA layer are timed once.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--parts ...]
                       [--no-beside] [--copy-calibration MIB]
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

PEAK = {"hbm_GBs": 8000.0, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0, "fp64_TFLOPs": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--parts", default="pair10,mpo8,batch,layer4")
    ap.add_argument("--no-beside", action="store_true",
                    help="skip the measurements beside the step (BF16 batch, plain loop, BF16 layer, measured peaks)")
    ap.add_argument("--batch-dtype", default="f32", choices=["f32", "bf16"],
                    help="core dtype of the batch part (bf16: the BF16 schedule as the timed part, for profiling it)")
    ap.add_argument("--layer-dtype", default="f32", choices=["f32", "bf16"],
                    help="arithmetic of the layer part (bf16: the BF16-MFMA option as the timed part, for profiling it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes five times (counter calibration)")
    ap.add_argument("--trace-batch", action="store_true",
                    help="only run the batch once with per-step clocks and print where its time goes")
    return ap.parse_args()


def trace_batch(ttc, batch_dtype):
    """One traced run of the 4096-pair batch (tt_batch_run_traced): each
    step's duration in shader cycles against its MFMA count (4 RT I QT
    (KC + PT) for the step's padded tiles: RT output row tiles, I mode
    indices, QT 16-wide slices of the second contracted bond, KC and PT the
    16-wide chunks of the first contracted bond and of the output columns),
    a least-squares fit cycles = fixed + per_mfma * MFMAs, and the cycles by
    MFMA-count range and by KC + PT."""
    import numpy as np
    import torch
    from ttgen import configs as C
    p16 = lambda n: (n + 15) // 16 * 16

    def y_first(rp, rn, pp, pn):
        return p16(pp) * p16(rn) * (p16(pn) + p16(rp)) < p16(rp) * p16(pn) * (p16(rn) + p16(pp))

    shapes = C.batch_pair_shapes(C.SEED_BATCH, 4096)
    pairs = C.gen_batch_torch(C.SEED_BATCH, shapes, "cuda", torch.bfloat16 if batch_dtype == "bf16" else torch.float32)
    plan = ttc.BatchPlan(pairs)
    inner, junc = plan.outputs()
    plan.run(inner, junc)
    torch.cuda.synchronize()
    _, _, per, steps = plan.run_traced(inner, junc)
    per, steps = per.numpy(), steps.numpy()
    mf, cyc, kp = [], [], []
    tail = 0.0
    for p, (sx, sy) in enumerate(shapes):
        n, prev = sx.order, per[p, 0]
        for j in range(n - 1):
            k = n - 1 - j
            rp, rn, pp, pn = sx.ranks[k], sx.ranks[k + 1], sy.ranks[k], sy.ranks[k + 1]
            ma, ka, nb, kb = (pp, pn, rp, rn) if y_first(rp, rn, pp, pn) else (rp, rn, pp, pn)
            mf.append(4 * (p16(ma) // 16) * sx.modes[k] * (p16(kb) // 16) * (p16(ka) // 16 + p16(nb) // 16))
            cyc.append(steps[p, j] - prev)
            kp.append(p16(ka) // 16 + p16(nb) // 16)
            prev = steps[p, j]
        tail += per[p, 1] - prev
    mf, cyc, kp = np.array(mf, float), np.array(cyc, float), np.array(kp)
    fit = np.linalg.lstsq(np.vstack([np.ones_like(mf), mf]).T, cyc, rcond=None)[0]
    wg = {}
    for p in range(len(shapes)):
        wg[int(per[p, 2])] = wg.get(int(per[p, 2]), 0.0) + float(per[p, 1] - per[p, 0])
    ranges = {}
    for lo, hi in ((0, 256), (256, 1024), (1024, 4096), (4096, 16384), (16384, 1 << 40)):
        m = (mf >= lo) & (mf < hi)
        if m.any():
            ranges[f"[{lo},{hi})"] = {"steps": int(m.sum()), "Gcycles": round(cyc[m].sum() / 1e9, 3),
                                      "cycles_per_mfma": round(cyc[m].sum() / mf[m].sum(), 1)}
    by_kp = {int(v): {"steps": int((kp == v).sum()),
                      "cycles_per_mfma": round(cyc[kp == v].sum() / mf[kp == v].sum(), 1)} for v in np.unique(kp)}
    print(json.dumps({"batch_trace": {"dtype": batch_dtype, "schedule": plan.config, "steps": len(mf),
                                      "fit_fixed_cycles": round(fit[0]), "fit_cycles_per_mfma": round(fit[1], 2),
                                      "step_Gcycles": round(cyc.sum() / 1e9, 3),
                                      "fixed_share": round(fit[0] * len(mf) / cyc.sum(), 3),
                                      "final_products_Gcycles": round(tail / 1e9, 3),
                                      "per_workgroup_Mcycles": {"mean": round(np.mean(list(wg.values())) / 1e6, 3),
                                                                "max": round(max(wg.values()) / 1e6, 3)},
                                      "by_mfma_count": ranges, "by_KC_plus_PT": by_kp}}))


# ------------------------------------------------------------- HBM traffic
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_digest(files):
    """SHA-256 over the sources a kernel is built from (recorded with its
    counter readings; a mismatch means the readings are stale)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter readings
    (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel calibration), or
    None when absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if kernel_source_digest(rec["sources"]) != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


# ------------------------------------------------------------- workload setup
def setup(parts, batch_dtype="f32"):
    import torch

    import paper_2109_00626_amd as ttc
    from ttgen import configs as C

    dev = torch.device("cuda:0")
    W = {}
    if "pair10" in parts:
        sx, sy = C.pair10_shapes()
        x = C.gen_tt_torch(C.SEED_PAIR10, 1, sx, dev, torch.float32)
        y = C.gen_tt_torch(C.SEED_PAIR10, 2, sy, dev, torch.float32)
        A = [C.gen_matrix_torch(C.SEED_PAIR10, 3 + n, 16, 16, dev, torch.float32) for n in range(10)]
        W["pair10"] = dict(x=x, y=y, A=A, sx=sx, sy=sy)
    if "mpo8" in parts:
        sw, sv = C.mpo8_shapes()
        W["mpo8"] = dict(w=C.gen_tt_torch(C.SEED_MPO8, 1, sw, dev, torch.bfloat16),
                         v=C.gen_tt_torch(C.SEED_MPO8, 2, sv, dev, torch.bfloat16), sw=sw, sv=sv)
    if "batch" in parts:
        shapes = C.batch_pair_shapes(C.SEED_BATCH, 4096)
        pairs = C.gen_batch_torch(C.SEED_BATCH, shapes, dev, torch.bfloat16 if batch_dtype == "bf16" else torch.float32)
        plan = ttc.BatchPlan(pairs)
        inner, junc = plan.outputs()
        W["batch"] = dict(shapes=shapes, pairs=pairs, plan=plan, inner=inner, junc=junc)
    if "layer4" in parts:
        s = C.layer4_shape()
        w = C.gen_tt_torch(C.SEED_LAYER, 1, s, dev, torch.float32)
        X = C.gen_matrix_torch(C.SEED_LAYER, 2, 8192, 4096, dev, torch.float32)
        T = C.gen_matrix_torch(C.SEED_LAYER, 3, 8192, 4096, dev, torch.float32)
        W["layer4"] = dict(w=w, X=X, T=T, s=s)
    torch.cuda.synchronize()
    return W


def run_part(name, W, ttc, prec_layer="f32"):
    if name == "pair10":
        d = W["pair10"]
        ttc.tt_contract_inner(d["x"], d["y"])
        ttc.tt_contract_modes(d["x"], d["y"], [0, 1, 2, 3, 4], "natural")
        ttc.tt_mode_n_product(d["x"], list(range(10)), d["A"])
        ttc.tt_contract_inner_bwd(d["x"], d["y"], 1.0)
    elif name == "mpo8":
        d = W["mpo8"]
        ttc.ttm_apply(d["w"], d["v"])
    elif name == "batch":
        d = W["batch"]
        d["plan"].run(d["inner"], d["junc"])
    elif name == "layer4":
        d = W["layer4"]
        Y = ttc.ttm_apply_dense(d["w"], d["X"], prec=prec_layer)
        _, dY = ttc.ttc_mse_loss(Y, d["T"])
        ttc.ttm_apply_dense_bwd(d["w"], d["X"], dY, prec=prec_layer)


CONTRACTIONS = {"pair10": 13, "mpo8": 1, "batch": 8192, "layer4": 2}


# ------------------------------------------------------------- algorithmic work
def algorithmic(W):
    """FLOPs and HBM bytes each part must move at minimum (inputs read once,
    outputs written once)."""
    out = {}
    if "pair10" in W:
        sx = W["pair10"]["sx"]
        R, I, N = 32, 16, 10
        # minimum-order sweep: 2*I*R^3*2 per interior step
        step = 2 * I * R * R * (R + R)
        inner = step * (N - 2) + 2 * 2 * I * R * R + 2 * R * R
        part = step * 4 + 2 * I * R * R
        nat_elems = 16384 + 3 * 16777216 + 524288 + 4 * 16384 + 512
        moden = sum(2 * sx.ranks[k] * 16 * 16 * sx.ranks[k + 1] for k in range(N))
        grad = 2 * inner + 2 * N * 2 * I * R * R * R * 2
        core_bytes = 4 * 2 * sum(sx.core_numel(k) for k in range(N))
        out["pair10"] = dict(flops=inner + part + moden + grad,
                             bytes=core_bytes * 4 + 4 * nat_elems + 4 * sum(sx.core_numel(k) for k in range(N)) * 3)
    if "mpo8" in W:
        sw, sv = W["mpo8"]["sw"], W["mpo8"]["sv"]
        fl = sum(2 * sw.ranks[k] * sw.modes[k] * sw.ranks[k + 1] * sv.ranks[k] * sv.ranks[k + 1] * sw.cols[k]
                 for k in range(8))
        outb = 4 * sum(sw.ranks[k] * sv.ranks[k] * sw.modes[k] * sw.ranks[k + 1] * sv.ranks[k + 1] for k in range(8))
        inb = 2 * (sw.numel() + sv.numel())
        out["mpo8"] = dict(flops=fl, bytes=outb + inb, out_bytes=outb)
    if "batch" in W:
        p = W["batch"]["plan"]
        out["batch"] = dict(flops=p.flops, bytes=p.bytes)
    if "layer4" in W:
        B, D = 8192, 4096
        gemm = 2.0 * B * D * D
        chain = 2.0 * (64 * 32 * 64 * 32 + 4096 * 32 * 64 * 32 + 262144 * 32 * 64)
        proj = 2.0 * (32 * 64 * 262144 + 262144 * 32 * 64 + 32 * 2048 * 4096 + 4096 * 32 * 2048 + 32 * 2048 * 64)
        fwd = gemm + chain
        out["layer4"] = dict(flops=fwd + 2 * gemm + chain + proj, fwd_flops=fwd, gemm_flops=gemm,
                             bytes=4.0 * B * D * 6)
    return out


# ------------------------------------------------------------- measured peaks
def measured_peaks(W, stream):
    """Reference rates measured on this GPU beside the nominal peaks: a
    plain 1 GiB device copy (bytes read + written per second) and a 1 GiB
    fill (bytes written per second) for HBM, and the vendor FP32 and BF16
    GEMMs (torch.mm, hipBLASLt) on the layer's forward shape for MFMA.  Neither is part of the path; they only give the
    achieved rates a second scale."""
    import torch

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    out = {}
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    ms = timed(lambda: dst.copy_(src), 10)
    out["hbm_copy_GBs"] = round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)
    # write-only stream (the natural-form lift and the MPO product are writes)
    ms = timed(lambda: dst.fill_(0.5), 10)
    out["hbm_fill_GBs"] = round(4 * n / (ms * 1e-3) / 1e9, 1)
    del src, dst
    if "layer4" in W:
        X = W["layer4"]["X"]
        g = torch.Generator(device="cuda:0")
        g.manual_seed(1)
        Wt = torch.randn(4096, 4096, dtype=torch.float32, device="cuda:0", generator=g)
        ms = timed(lambda: torch.mm(X, Wt), 5)
        out["fp32_gemm_TFLOPs"] = round(2.0 * X.shape[0] * 4096 * 4096 / (ms * 1e-3) / 1e12, 2)
        Xh, Wh = X.to(torch.bfloat16), Wt.to(torch.bfloat16)
        ms = timed(lambda: torch.mm(Xh, Wh), 5)
        out["bf16_gemm_TFLOPs"] = round(2.0 * X.shape[0] * 4096 * 4096 / (ms * 1e-3) / 1e12, 2)
        del Wt, Xh, Wh
    torch.cuda.synchronize()
    return out


# ------------------------------------------------------------- Example 2
EX2_DIMS = [(20, 20, 20), (20, 20, 20, 5), (20, 20, 20, 5, 4)]
SEED_EX2 = 210900626 + 7


def example2_inputs(dims, device, dtype):
    """Gaussian N(0, 1) tensors X and Y of shape `dims` (the paper's Example 2)."""
    from ttgen import configs as C
    n = int(math.prod(dims))
    X = C.gen_matrix_torch(SEED_EX2, 1, 1, n, device, dtype).reshape(dims)
    Y = C.gen_matrix_torch(SEED_EX2, 2, 1, n, device, dtype).reshape(dims)
    return X, Y


def example2_gpu(ttc, reps=3):
    """Example 2 on the GPU: TTCP of X x_1^1 Y from dense inputs, i.e. TT-SVD
    of both (Algorithm 1, eps = 0) and the contraction of their first cores
    (the junction K and the free cores), wall time per run (the TT-SVD reads
    singular values back once per split)."""
    import torch
    out = {}
    for dims in EX2_DIMS:
        X, Y = example2_inputs(dims, "cuda", torch.float64)
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gx = ttc.tt_svd(X)
            gy = ttc.tt_svd(Y)
            K = ttc.tt_contract_pairs(gx, gy, [0], [0], "junction")
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out["x".join(map(str, dims))] = {"ttcp_ms": round(1e3 * sorted(ts[1:])[len(ts[1:]) // 2], 3),
                                        "ranks_x": [int(g.shape[0]) for g in gx] + [1],
                                        "K_shape": [int(K.shape[0]), int(K.shape[1])]}
    return out


# ------------------------------------------------------------- CPU baseline
def cpu_baseline(W, n_contr, budget_s=20.0):
    """The FP64 oracle as it is, on a bounded sample of each part, each part's
    time scaled to its full size; returns TT contractions/s of the step."""
    import numpy as np
    import torch

    from oracle import tt_oracle as O

    def np_cores(ts):
        return [t.detach().to(torch.float64).cpu().numpy() for t in ts]

    est, sample = {}, []
    t_all = time.perf_counter()
    if "pair10" in W:
        d = W["pair10"]
        x, y = np_cores(d["x"]), np_cores(d["y"])
        A = [a.double().cpu().numpy() for a in d["A"]]
        t0 = time.perf_counter()
        O.inner_lr(x, y)
        O.contract_natural(x, y, [0, 1, 2, 3, 4])
        z = x
        for n in range(10):
            z = O.mode_n_tt(z, n, A[n])
        O.inner_grad(x, y)
        est["pair10"] = time.perf_counter() - t0
        sample.append("pair10 in full")
    if "mpo8" in W:
        d = W["mpo8"]
        w, v = np_cores(d["w"]), np_cores(d["v"])
        fl = [w[k].size * v[k].shape[0] * v[k].shape[2] for k in range(8)]
        done, t1 = [], 0.0
        for k in (3, 4, 2, 5, 1, 6, 0, 7):
            t0 = time.perf_counter()
            O.mpo_tt([w[k]], [v[k]])
            t1 += time.perf_counter() - t0
            done.append(k)
            if t1 >= budget_s * 0.2:
                break
        est["mpo8"] = t1 * sum(fl) / sum(fl[k] for k in done)
        sample.append(f"mpo8 cores {sorted(k + 1 for k in done)} of 8, scaled by FLOPs")
    if "batch" in W:
        d = W["batch"]
        plan = d["plan"]
        rs = np.random.RandomState(0)
        order = rs.permutation(len(d["pairs"]))

        def pair_flops(sx, sy):
            return sum(2 * sx.ranks[k] * sx.modes[k] * sx.ranks[k + 1] * (sy.ranks[k] + sy.ranks[k + 1]) * sy.ranks[k + 1]
                       for k in range(sx.order))

        # random pairs until the part's share of the budget is spent
        fl, t1, n_done = 0, 0.0, 0
        for p in order:
            x, y = np_cores(d["pairs"][p][0]), np_cores(d["pairs"][p][1])
            t0 = time.perf_counter()
            O.inner_lr(x, y)
            O.sweep_rl(x, y, downto=len(x) - 2)
            t1 += time.perf_counter() - t0
            fl += pair_flops(*d["shapes"][p])
            n_done += 1
            if t1 >= budget_s * 0.4:
                break
        full = sum(pair_flops(sx, sy) for sx, sy in d["shapes"])
        est["batch"] = t1 * full / fl
        sample.append(f"batch: {n_done} random pairs of 4096, scaled by FLOPs")
    if "layer4" in W:
        d = W["layer4"]
        w = np_cores(d["w"])
        rows = 512
        X = d["X"][:rows].double().cpu().numpy()
        T = d["T"][:rows].double().cpu().numpy()
        t0 = time.perf_counter()
        Wd = O.mpo_full(w)
        t_fixed = time.perf_counter() - t0
        t0 = time.perf_counter()
        Y = X @ Wd.T
        L, dY = O.mse_loss(Y, T)
        dX = dY @ Wd
        dW = dY.T @ X
        t_rows = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.mpo_core_grads_from_dense(w, dW)
        t_fixed += time.perf_counter() - t0
        est["layer4"] = t_fixed + t_rows * (8192 / rows)
        sample.append(f"layer4: {rows} of 8192 rows (row-proportional work scaled by {8192 // rows}, "
                      "reconstruction and projection once)")
    # Example 2 on the host: the oracle's dense eq. (8) and its TTCP
    # (Algorithm 2 with TT-SVD), on the same Gaussian tensors
    ex2 = {}
    for dims in EX2_DIMS:
        X, Y = (t.numpy() for t in example2_inputs(dims, "cpu", torch.float64))
        t0 = time.perf_counter()
        O.tcp(X, Y, 0, 0)
        t1 = time.perf_counter()
        O.ttcp(X, Y, 0, 0)
        t2 = time.perf_counter()
        ex2["x".join(map(str, dims))] = {"dense_tcp_ms": round(1e3 * (t1 - t0), 3), "ttcp_ms": round(1e3 * (t2 - t1), 3)}
    total = sum(est.values())
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(i.get("num_threads", 1) for i in info)
    except Exception:
        pass
    return {
        "value": n_contr / total if total > 0 else None,
        "unit": "TT contractions/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "; ".join(sample) + f"; measured {time.perf_counter() - t_all:.1f} s, estimated full step "
                                      f"{total:.2f} s",
        "est_seconds_per_part": {k: round(v, 4) for k, v in est.items()},
        "example2": ex2,
    }


# ------------------------------------------------------------- main
def main():
    import numpy as np

    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(how the path would shard is described in the design notes)"}))
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 4 * n, "launches": 5}))
        return

    import paper_2109_00626_amd as ttc

    if args.trace_batch:
        trace_batch(ttc, args.batch_dtype)
        return

    parts = [p for p in args.parts.split(",") if p]
    W = setup(parts, args.batch_dtype)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        for p in parts:
            run_part(p, W, ttc, args.layer_dtype)
    torch.cuda.synchronize()
    ev = {p: [] for p in parts}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for p in parts:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            run_part(p, W, ttc, args.layer_dtype)
            b.record(stream)
            ev[p].append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    part_ms = {p: sum(a.elapsed_time(b) for a, b in ev[p]) / args.steps for p in parts}
    ms_step = 1e3 * wall / args.steps
    n_contr = sum(CONTRACTIONS[p] for p in parts)
    alg = algorithmic(W)

    # the layer forward alone (its GEMM is the largest launch of the step)
    fwd_ms = None
    if "layer4" in parts:
        d = W["layer4"]
        evs = []
        for _ in range(max(3, args.steps)):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ttc.ttm_apply_dense(d["w"], d["X"], prec=args.layer_dtype)
            b.record(stream)
            evs.append((a, b))
        torch.cuda.synchronize()
        fwd_ms = sorted(a.elapsed_time(b) for a, b in evs)[len(evs) // 2]

    parts_out = {}
    for p in parts:
        ms = part_ms[p]
        o = {"ms": round(ms, 4), "contractions": CONTRACTIONS[p],
             "TFLOPs": round(alg[p]["flops"] / (ms * 1e-3) / 1e12, 3),
             "GBs": round(alg[p]["bytes"] / (ms * 1e-3) / 1e9, 1)}
        parts_out[p] = o
    dominant = max(parts, key=lambda p: part_ms[p])
    # roofline of the dominant part's main kernel
    if dominant == "layer4" and args.layer_dtype == "bf16":
        ach = alg["layer4"]["fwd_flops"] / (fwd_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "gemm16_kernel (BF16 16x16x32 MFMA), measured as the whole forward call "
                                            "(W rebuild, operand conversions, product)",
                "achieved": round(ach, 2), "peak": PEAK["bf16_TFLOPs"], "unit": "TFLOP/s",
                "frac": round(ach / PEAK["bf16_TFLOPs"], 4), "traffic": recorded_traffic("gemm16_kernel"),
                "per_launch": "2 * 8192 * 4096 * 4096 FLOP (+ 1.1 GFLOP core chain)"}
    elif dominant == "layer4":
        gemm_ms = fwd_ms
        ach = alg["layer4"]["fwd_flops"] / (gemm_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "gemm_kernel (FP32 32x32x2 MFMA), measured as the whole forward call",
                "achieved": round(ach, 2), "peak": PEAK["fp32_TFLOPs"], "unit": "TFLOP/s",
                "frac": round(ach / PEAK["fp32_TFLOPs"], 4), "traffic": recorded_traffic("gemm_kernel"),
                "per_launch": "2 * 8192 * 4096 * 4096 FLOP (+ 1.1 GFLOP core chain)"}
    elif dominant == "batch":
        ms = part_ms["batch"]
        ach = alg["batch"]["bytes"] / (ms * 1e-3) / 1e9
        cfg = W["batch"]["plan"].config
        kname = {"lds": "batch_lds_kernel", "lds1": "batch_lds_kernel_inplace", "lds1b": "batch_lds_kernel_b16",
                 "persistent": "batch_kernel", "levels": "level_kernel"}[cfg["mode"]]
        roof = {"bound": "hbm", "kernel": kname, "schedule": cfg, "achieved": round(ach, 1),
                "peak": PEAK["hbm_GBs"], "unit": "GB/s", "frac": round(ach / PEAK["hbm_GBs"], 4),
                "traffic": recorded_traffic(f"{kname}/{cfg['threads']}") if cfg["mode"] in ("lds", "lds1", "lds1b") else None,
                "per_launch": "all 4096 pairs: every core read once, 4096 FP64 scalars and the junctions written"}
    else:
        ms = part_ms[dominant]
        ach = alg[dominant]["bytes"] / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dominant, "achieved": round(ach, 1), "peak": PEAK["hbm_GBs"],
                "unit": "GB/s", "frac": round(ach / PEAK["hbm_GBs"], 4), "traffic": None}

    if not args.no_beside:
        mp = measured_peaks(W, stream)
        if roof["unit"] == "GB/s" and "hbm_copy_GBs" in mp:
            roof["measured_peak"] = {"value": mp["hbm_copy_GBs"], "what": "1 GiB device copy, bytes read + written"}
            roof["frac_of_measured"] = round(roof["achieved"] / mp["hbm_copy_GBs"], 4)
        elif roof["unit"] == "TFLOP/s" and "fp32_gemm_TFLOPs" in mp:
            roof["measured_peak"] = {"value": mp["fp32_gemm_TFLOPs"],
                                     "what": "vendor FP32 GEMM (torch.mm) on the same 8192 x 4096 x 4096 shape"}
            roof["frac_of_measured"] = round(roof["achieved"] / mp["fp32_gemm_TFLOPs"], 4)

    beside = {}
    if not args.no_beside:
        beside["measured_peaks"] = mp
    if "batch" in parts and not args.no_beside and args.batch_dtype == "f32":
        d = W["batch"]
        plan = d["plan"]

        def timeit(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        plain_ms = timeit(lambda: plan.run(d["inner"], d["junc"], plain=True), reps=2)
        beside["batch_fp32"] = {"batched_ms": round(part_ms["batch"], 4), "plain_loop_ms": round(plain_ms, 4),
                                "contractions_per_s": round(8192 / (part_ms["batch"] * 1e-3), 1),
                                "GBs": parts_out["batch"]["GBs"], "TFLOPs": parts_out["batch"]["TFLOPs"],
                                "algorithmic_GB": round(plan.bytes / 1e9, 3),
                                "algorithmic_GFLOP": round(plan.flops / 1e9, 3),
                                "frac_of_copy": round(parts_out["batch"]["GBs"] / mp["hbm_copy_GBs"], 4)}
        from ttgen import configs as C
        pairs_bf = C.gen_batch_torch(C.SEED_BATCH, d["shapes"], "cuda", torch.bfloat16)
        plan_bf = ttc.BatchPlan(pairs_bf)
        ib, jb = plan_bf.outputs()
        bf_ms = timeit(lambda: plan_bf.run(ib, jb), reps=5)
        beside["batch_bf16"] = {"batched_ms": round(bf_ms, 4),
                                "contractions_per_s": round(8192 / (bf_ms * 1e-3), 1),
                                "GBs": round(plan_bf.bytes / (bf_ms * 1e-3) / 1e9, 1),
                                "TFLOPs": round(plan_bf.flops / (bf_ms * 1e-3) / 1e12, 3),
                                "algorithmic_GB": round(plan_bf.bytes / 1e9, 3),
                                "frac_of_copy": round(plan_bf.bytes / (bf_ms * 1e-3) / 1e9 / mp["hbm_copy_GBs"], 4),
                                "schedule": plan_bf.config}
        del pairs_bf, plan_bf, ib, jb
    if "layer4" in parts and not args.no_beside:
        d = W["layer4"]

        def layer(prec):
            Y = ttc.ttm_apply_dense(d["w"], d["X"], prec=prec)
            _, dY = ttc.ttc_mse_loss(Y, d["T"])
            ttc.ttm_apply_dense_bwd(d["w"], d["X"], dY, prec=prec)

        for prec in ("bf16",):
            layer(prec)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(3):
                layer(prec)
            b.record(stream)
            torch.cuda.synchronize()
            beside[f"layer4_{prec}_fwd_bwd_ms"] = round(a.elapsed_time(b) / 3, 4)
        beside["layer4_f32_fwd_bwd_ms"] = round(part_ms["layer4"], 4)
        beside["layer4_f32_fwd_ms"] = round(fwd_ms, 4)
        # the core-by-core schedule (the method applied to the batch): one
        # GEMM per core, 4x the FLOPs of the dense schedule on this shape;
        # forward + backward keep the forward's intermediates for the
        # backward (schedule cores_saved, one workspace for both calls)
        cws = torch.empty(max(ttc.ttm_apply_dense_query(d["w"], 8192, p, "cores_saved", backward=True)
                              for p in ("f32", "bf16")), dtype=torch.uint8, device=d["X"].device)

        def cores(bwd, prec):
            if not bwd:
                ttc.ttm_apply_dense(d["w"], d["X"], sched="cores", prec=prec)
                return
            Y = ttc.ttm_apply_dense(d["w"], d["X"], sched="cores_saved", prec=prec, ws=cws)
            _, dY = ttc.ttc_mse_loss(Y, d["T"])
            ttc.ttm_apply_dense_bwd(d["w"], d["X"], dY, sched="cores_saved", prec=prec, ws=cws)

        for bwd, prec, key in ((False, "f32", "layer4_cores_f32_fwd_ms"), (True, "f32", "layer4_cores_f32_fwd_bwd_ms"),
                               (True, "bf16", "layer4_cores_bf16_fwd_bwd_ms")):
            cores(bwd, prec)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            cores(bwd, prec)
            b.record(stream)
            torch.cuda.synchronize()
            beside[key] = round(a.elapsed_time(b), 4)
        # executed FLOPs: forward = sum over cores of 2 |P_k| |Q_k| (J_k R_k) (I_k R_{k+1})
        sh = d["s"]
        fl = 0.0
        for k in range(4):
            P = 8192 * int(np.prod(sh.cols[k + 1:])) if k < 3 else 8192
            Q = int(np.prod(sh.modes[:k])) if k > 0 else 1
            fl += 2.0 * P * Q * sh.cols[k] * sh.ranks[k] * sh.modes[k] * sh.ranks[k + 1]
        beside["layer4_cores_f32_fwd_TFLOPs"] = round(fl / (beside["layer4_cores_f32_fwd_ms"] * 1e-3) / 1e12, 2)
        # forward + backward executes three products of the forward's size per
        # core (forward, input gradient, core gradient)
        beside["layer4_cores_f32_fwd_bwd_TFLOPs"] = round(3 * fl / (beside["layer4_cores_f32_fwd_bwd_ms"] * 1e-3) / 1e12,
                                                         2)

    # a middle block of the order-10 pair (X's modes 4-7 with Y's, eq. (8)
    # once per pair): the two-sided transfer, executed FLOPs of its products
    if not args.no_beside and "pair10" in W:
        d = W["pair10"]
        mid = [3, 4, 5, 6]
        f = lambda: ttc.tt_contract_pairs(d["x"], d["y"], mid, mid, "junction")
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            f()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 20
        sx, sy = d["sx"], d["sy"]
        a0, g0 = sx.ranks[mid[0]], sy.ranks[mid[0]]
        fl = 2.0 * a0 * g0 * sx.ranks[mid[0] + 1] * sy.ranks[mid[0] + 1] * sx.modes[mid[0]]
        for k in mid[1:]:
            ka1, kg1, nm, kb, kd = sx.ranks[k], sy.ranks[k], sx.modes[k], sx.ranks[k + 1], sy.ranks[k + 1]
            fl += 2.0 * a0 * g0 * (kg1 * nm * kb * ka1 + kb * kd * kg1 * nm)
        beside["pairs_middle_fp32"] = {"modes": [m + 1 for m in mid], "ms": round(ms, 4),
                                       "GFLOP": round(fl / 1e9, 3), "TFLOPs": round(fl / (ms * 1e-3) / 1e12, 2)}

    # the TT-method kernels against their own rooflines (the step's dominant
    # kernel above is the layer's dense-schedule GEMM)
    if not args.no_beside:
        mr = {}

        def hbm(name, kernel, gbs, traffic=None):
            mr[name] = {"kernel": kernel, "bound": "hbm", "achieved_GBs": round(gbs, 1),
                        "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": traffic}

        if "batch_fp32" in beside:
            bc = W["batch"]["plan"].config
            hbm("batch_fp32", "batch_lds_kernel (FP32 cores, FP32 MFMA steps)", beside["batch_fp32"]["GBs"],
                recorded_traffic(f"batch_lds_kernel_inplace/{bc['threads']}") if bc["mode"] == "lds1" else None)
        if "batch_bf16" in beside:
            hbm("batch_bf16", "batch_lds_kernel (BF16 cores, " + beside["batch_bf16"]["schedule"]["mode"] + ")",
                beside["batch_bf16"]["GBs"])
        if "mpo8" in parts:
            hbm("mpo8", "mpo16_kernel (BF16 MFMA, write stream)", parts_out["mpo8"]["GBs"],
                recorded_traffic("mpo16_kernel"))
        if "layer4_cores_f32_fwd_bwd_TFLOPs" in beside:
            t = beside["layer4_cores_f32_fwd_bwd_TFLOPs"]
            mr["layer4_cores_fwd_bwd"] = {"kernel": "gemm_kernel (FP32 MFMA), one product per core and direction",
                                          "bound": "mfma", "achieved_TFLOPs": t,
                                          "frac": round(t / PEAK["fp32_TFLOPs"], 4)}
            t16 = beside["layer4_cores_f32_fwd_bwd_TFLOPs"] * beside["layer4_cores_f32_fwd_bwd_ms"] / \
                beside["layer4_cores_bf16_fwd_bwd_ms"]
            mr["layer4_cores_bf16_fwd_bwd"] = {"kernel": "gemm_kernel (BF16 MFMA, FP32 operands rounded while staged)",
                                               "bound": "mfma", "achieved_TFLOPs": round(t16, 2),
                                               "frac": round(t16 / PEAK["bf16_TFLOPs"], 4)}
        if "pairs_middle_fp32" in beside:
            t = beside["pairs_middle_fp32"]["TFLOPs"]
            mr["pairs_middle_fp32"] = {"kernel": "gemm_kernel batched over the transfer rows (FP32 MFMA), the whole call",
                                       "bound": "mfma", "achieved_TFLOPs": t, "frac": round(t / PEAK["fp32_TFLOPs"], 4)}
        beside["method_rooflines"] = mr

    if not args.no_beside:
        beside["example2"] = example2_gpu(ttc)

    line = {
        "metric": "TT contractions/s + achieved GB/s or TFLOP/s vs roofline; fwd+bwd ms, plain vs batched",
        "value": round(n_contr / (ms_step * 1e-3), 2),
        "unit": "TT contractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (mpo8: bf16 in, f32 acc)" if args.batch_dtype == "f32" else "f32 (mpo8, batch: bf16 in, f32 acc)",
        "data": "synthetic (seeded generator; shapes and distributions of the five workloads)",
        "config": {"workload": "tt-hot-path: " + "+".join(parts) + (" (batch with BF16 cores)" if args.batch_dtype == "bf16" else ""),
                   "contractions_per_step": {p: CONTRACTIONS[p] for p in parts},
                   "parallelism": "single GPU"},
        "roofline": roof,
        "parts": parts_out,
        "beside": beside,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(W, n_contr)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
