"""Throughput of the tall & skinny products on one MI355X.

One step is one pass of the plain width sweep: TSMTTSM (C = A^T B) and TSMM
(B = A C) in real (D) and complex (Z) double precision, K = 2^24 rows,
(M, N) in {(1,1), (2,2), (4,4), (8,8), (16,16), (32,32), (64,64), (32,8), (8,32)}:
36 calls on inputs already resident in HBM (seeded uniform(-1, 1) data,
generated on the device).  The value is the sweep's algorithmic bytes per
second (Eq. 1 of the paper: every element of A, B and C moves once); the JSON
line also carries each call's GB/s, GFLOP/s and fraction of the
min(HBM, FP64) roofline, the roofline record of the dominant kernel and the
CPU oracle timed on a bounded sample of the same sweep.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --all-widths      # every square width 1..64 instead (one JSON line each)
    python bench.py --all-widths --vendor   # ... with torch.matmul (rocBLAS / hipBLASLt) beside each
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12        # B/s, MI355X HBM3E (published)
FP64_PEAK = 78.6e12      # flop/s, MI355X FP64 vector and matrix (published)
METRIC = "TSMTTSM/TSMM GB/s & % of roofline vs width; mixed/batched speedup vs FP64"
WIDTHS = [(1, 1), (2, 2), (4, 4), (8, 8), (16, 16), (32, 32), (64, 64), (32, 8), (8, 32)]
FLUSH_ORDER = [(64, 64), (1, 1), (32, 32), (2, 2), (16, 16), (4, 4), (32, 8), (8, 8), (8, 32)]
K_SWEEP = 1 << 24


def algorithmic(op, cplx, K, M, N, beta=0.0):
    """Bytes and flops one call must move / compute (Eq. 1: A, B and C each
    cross the memory interface once; 2MNK flops, 4x for complex)."""
    s = 16 if cplx else 8
    byts = s * (K * M + K * N + M * N)
    if op == "tsmm" and beta != 0.0:
        byts += s * K * N
    flops = (8 if cplx else 2) * M * N * K
    return byts, flops


def roofline_time(byts, flops, bw=HBM_PEAK, peak=FP64_PEAK):
    return max(byts / bw, flops / peak)


def measure_bs(torch, src, dst, nbytes=8 << 30, reps=5):
    """Achievable bandwidth b_s on this GPU with the library's probes (the
    paper's read-only sum and read+write stream, Section 1.6): the median of
    `reps` timed passes over `nbytes` (far beyond the 256 MB Infinity Cache).
    'copy' counts read plus written bytes."""
    from paper_1905_03136_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    out = {}
    for kind in ("read", "copy"):
        times = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            if kind == "read":
                _lib.check(_lib.tsg_stream_read(src.data_ptr(), nbytes, s))
            else:
                _lib.check(_lib.tsg_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, s))
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        t = sorted(times[1:])[reps // 2]
        out[kind] = (nbytes if kind == "read" else 2 * nbytes) / t
    return out


def time_call(torch, fn, reps=3, warmup=1):
    """Median device time of fn() over `reps` runs (events on the current stream)."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return sorted(ts)[len(ts) // 2]


def precision_form(torch, api, inputs, dev, K=1 << 25, widths=(8, 32, 64)):
    """Speedup of binary32 storage (exact products, binary64 accumulation)
    over binary64 storage for both products, real and complex, at K = 2^25."""
    out = []
    for cplx in (False, True):
        t64 = torch.complex128 if cplx else torch.float64
        t32 = torch.complex64 if cplx else torch.float32
        A = inputs.device_uniform(K, 64, 7, inputs.STREAM_A, cplx, dev)
        B = inputs.device_uniform(K, 64, 7, inputs.STREAM_B, cplx, dev)
        A32, B32 = A.to(t32), B.to(t32)
        X = inputs.device_uniform(64, 64, 7, inputs.STREAM_C, cplx, dev)
        for w in widths:
            a64 = A.reshape(-1)[:K * w].view(K, w)
            b64 = B.reshape(-1)[:K * w].view(K, w)
            a32 = A32.reshape(-1)[:K * w].view(K, w)
            b32 = B32.reshape(-1)[:K * w].view(K, w)
            x = X[:w, :w].contiguous()
            rec = {"dtype": "Z" if cplx else "D", "M": w, "N": w, "K": K}
            for op in ("tsmttsm", "tsmm"):
                if op == "tsmttsm":
                    f64 = (lambda: api.tsmttsm(a64, b64))
                    f32 = (lambda: api.tsmttsm(a32, b32))
                else:
                    f64 = (lambda: api.tsmm(a64, x, out=b64))
                    f32 = (lambda: api.tsmm(a32, x, out=b32))
                t_64 = time_call(torch, f64)
                t_32 = time_call(torch, f32)
                s = 16 if cplx else 8
                rec[op] = {"us_fp64": round(t_64 * 1e6, 1), "us_fp32": round(t_32 * 1e6, 1),
                           "speedup": round(t_64 / t_32, 3),
                           "GBps_fp32": round((s // 2) * K * 2 * w / t_32 / 1e9, 1),
                           "kernel_fp32": api.kernel_name(op, t32, w, w)}
            out.append(rec)
        del A, B, A32, B32
        torch.cuda.empty_cache()
    return {"note": "binary32 / complex64 storage of A and B (values widened exactly, products exact, "
                    "binary64 accumulation and reduction) against binary64 / complex128 storage; arithmetic "
                    "error against the binary64 oracle on the stored values is at the binary64 level "
                    "(tests check <= 1e-12 for TSMTTSM, one binary32 rounding for TSMM outputs)",
            "widths": out}


def batched_form(torch, api, inputs, dev, reps=5):
    """64 block-orthogonalisation steps (C_i = V_i^T W_i, W_i -= V_i C_i),
    K_i log-uniform in [2^16, 2^22], M_i in {4,8,16,32,64}, N_i in {1,4,8,16}:
    one persistent launch replayed from its graph, against the same work as
    128 separate library calls (64 TSMTTSM + 64 TSMM updates) on one stream,
    and against those calls captured in one graph.  V_i is uniform(-1, 1)
    scaled by sqrt(3 / K_i) (columns of unit expected norm, nearly orthogonal)
    so that repeated in-place steps keep W bounded; the time does not depend
    on the values."""
    from paper_1905_03136_amd import _lib
    shapes = inputs.batched_instances(64, seed=0)
    pairs, Cs = [], []
    for i, (K, M, N) in enumerate(shapes):
        V = inputs.device_uniform(K, M, 100 + i, inputs.STREAM_V0, False, dev)
        V.mul_((3.0 / K) ** 0.5)
        W = inputs.device_uniform(K, N, 100 + i, inputs.STREAM_W0, False, dev)
        pairs.append((V, W))
        Cs.append(torch.empty((M, N), dtype=torch.float64, device=dev))
    byts = sum(8 * K * (2 * M + 3 * N) for K, M, N in shapes)
    ideal = sum(8 * K * (M + 2 * N) for K, M, N in shapes)
    flops = sum(4 * K * M * N for K, M, N in shapes)
    W0 = [w.clone() for _, w in pairs]

    def separate():
        for (V, W), C in zip(pairs, Cs):
            api.tsmttsm(V, W, out=C)
            api.tsmm(V, C, out=W, alpha=-1.0, beta=1.0)

    plan = api.OrthPlan(pairs)
    t_persist = time_call(torch, plan.launch, reps=reps, warmup=2)
    plan.check()
    t_sep = time_call(torch, separate, reps=reps, warmup=2)
    # the separate calls captured into one graph (workspaces reserved by the warm-up on the capture stream)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        separate()
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        separate()
    t_graph = time_call(torch, g.replay, reps=reps, warmup=2)
    # agreement of the two paths from the same W (different summation orders)
    for (_, w), w0 in zip(pairs, W0):
        w.copy_(w0)
    plan.launch()
    plan.check()
    C_p = [c.clone() for c in plan.C]
    W_p = [w.clone() for _, w in pairs]
    for (_, w), w0 in zip(pairs, W0):
        w.copy_(w0)
    separate()
    torch.cuda.synchronize()
    rel_C = max(float((a - b).norm() / b.norm().clamp_min(1e-300)) for a, b in zip(C_p, Cs))
    rel_W = max(float((a - w).norm() / w.norm().clamp_min(1e-300)) for a, (_, w) in zip(W_p, pairs))
    plan.close()
    del g
    return {"instances": 64, "rows": sum(k for k, _, _ in shapes),
            "algorithmic_bytes": byts, "cache_ideal_bytes": ideal, "flops": flops,
            "us_persistent_graph": round(t_persist * 1e6, 1), "us_128_launches": round(t_sep * 1e6, 1),
            "us_128_launches_graph": round(t_graph * 1e6, 1),
            "speedup_vs_launches": round(t_sep / t_persist, 3),
            "speedup_vs_launch_graph": round(t_graph / t_persist, 3),
            "GBps_persistent": round(byts / t_persist / 1e9, 1),
            "roof_frac_persistent": round(byts / t_persist / HBM_PEAK, 4),
            "GBps_persistent_cache_ideal": round(ideal / t_persist / 1e9, 1),
            "GBps_128_launches": round(byts / t_sep / 1e9, 1),
            "max_rel_diff_C": rel_C, "max_rel_diff_W": rel_W,
            "note": "bytes = sum 8 K (2M + 3N) (phase 1 reads V and W; phase 2 reads V and W and writes W); "
                    "cache-ideal sum 8 K (M + 2N); rel diffs are normwise between the persistent and the "
                    "separate-launch results from the same inputs"}


def cpu_baseline(K_sample):
    import numpy as np

    import oracle
    from paper_1905_03136_amd import inputs
    oracle.build()
    threads = oracle.max_threads()
    total_bytes = 0
    t_total = 0.0
    for cplx in (False, True):
        A = inputs.host_uniform(K_sample, 64, 0, inputs.STREAM_A, cplx)
        B = inputs.host_uniform(K_sample, 64, 0, inputs.STREAM_B, cplx)
        Xfull = inputs.host_uniform(64, 64, 0, inputs.STREAM_C, cplx)
        for (M, N) in WIDTHS:
            a = np.ascontiguousarray(A[:, :M])
            b = np.ascontiguousarray(B[:, :N])
            X = np.ascontiguousarray(Xfull[:M, :N])
            t0 = time.perf_counter()
            oracle.tsmttsm(a, b)
            t1 = time.perf_counter()
            oracle.tsmm(a, X)
            t2 = time.perf_counter()
            t_total += t2 - t0
            for op in ("tsmttsm", "tsmm"):
                total_bytes += algorithmic(op, cplx, K_sample, M, N)[0]
    return {"value": total_bytes / t_total / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "the same 36-call sweep (TSMTTSM+TSMM, D and Z, 9 widths) at K=%d rows instead of "
                      "2^24; plain binary64 triple loop, threads over output rows; %.1f s" % (K_sample, t_total),
            "seconds": t_total, "cpu": platform.processor() or platform.machine()}


def all_widths(torch, api, inputs, dev, K=K_SWEEP, reps=3, vendor=False):
    """Every square width M = N = 1..64, D and Z, both products at K rows:
    median time of `reps` calls (one width at a time, exact-size operands)
    and the fraction of the spec roofline; one JSON line per width, then a
    summary line with the mean and the minimum fraction per (dtype, op).
    With `vendor`, the same products through torch.matmul (rocBLAS /
    hipBLASLt GEMMs: A^T B as a transposed view times B, A C) are timed on
    the same operands beside ours -- the vendor-library context of the
    paper's library comparison (Section 1.5), measured on this GPU."""
    rows = []
    for cplx in (False, True):
        for w in range(1, 65):
            A = inputs.device_uniform(K, w, w, inputs.STREAM_A, cplx, dev)
            B = inputs.device_uniform(K, w, w, inputs.STREAM_B, cplx, dev)
            X = inputs.device_uniform(w, w, w, inputs.STREAM_C, cplx, dev)
            Co = torch.empty((w, w), dtype=A.dtype, device=dev)
            rec = {"dtype": "Z" if cplx else "D", "M": w, "N": w, "K": K}
            for op, fn in (("tsmttsm", lambda: api.tsmttsm(A, B, out=Co)), ("tsmm", lambda: api.tsmm(A, X, out=B))):
                t = time_call(torch, fn, reps=reps, warmup=1)
                byts, flops = algorithmic(op, cplx, K, w, w)
                roof = max(byts / HBM_PEAK, flops / FP64_PEAK)
                rec[op] = {"us": round(t * 1e6, 1), "roof_frac": round(roof / t, 4),
                           "kernel": api.kernel_name(op, A.dtype, w, w)}
                if vendor:
                    vfn = (lambda: torch.matmul(A.t(), B, out=Co)) if op == "tsmttsm" else \
                        (lambda: torch.matmul(A, X, out=B))
                    tv = time_call(torch, vfn, reps=reps, warmup=1)
                    rec[op].update(vendor_us=round(tv * 1e6, 1), vendor_roof_frac=round(roof / tv, 4),
                                   speedup_vs_vendor=round(tv / t, 3))
            print(json.dumps(rec), flush=True)
            rows.append(rec)
            del A, B, X, Co
    summary = {}
    for dt in ("D", "Z"):
        for op in ("tsmttsm", "tsmm"):
            f = [r[op]["roof_frac"] for r in rows if r["dtype"] == dt]
            summary["%s_%s" % (dt, op)] = {"mean": round(sum(f) / len(f), 4), "min": min(f)}
            if vendor:
                v = [r[op]["vendor_roof_frac"] for r in rows if r["dtype"] == dt]
                sp = [r[op]["speedup_vs_vendor"] for r in rows if r["dtype"] == dt]
                summary["%s_%s" % (dt, op)].update(
                    vendor_mean=round(sum(v) / len(v), 4), vendor_min=min(v), vendor_max=max(v),
                    speedup_min=min(sp), speedup_median=sorted(sp)[len(sp) // 2])
    print(json.dumps({"all_widths_summary": summary}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    # 3 * 2^22 rows: the 36 calls of the sweep move 201 GB at that K, about 13 s
    # of oracle work on 16 host threads (15.4 GB/s measured at 2^23 rows);
    # inputs of at most 12.9 GB per matrix
    ap.add_argument("--cpu-sample", type=int, default=3 << 22, help="rows of the oracle sample (0 = skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the post-run spot check")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision / batched form measurements")
    ap.add_argument("--all-widths", action="store_true",
                    help="instead of the bench step: every square width 1..64 (D, Z, both products), one JSON line each")
    ap.add_argument("--vendor", action="store_true",
                    help="with --all-widths: also time torch.matmul (rocBLAS / hipBLASLt) on the same operands")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the products run on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_03136_amd import api, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.all_widths:
        all_widths(torch, api, inputs, dev, vendor=a.vendor)
        return
    print("[bench] allocating and generating inputs", file=sys.stderr, flush=True)
    K = K_SWEEP
    # Every width has its own exact-size A (K x M) and B (K x N), as a caller's
    # matrices would be (134 GB in all); TSMTTSM reads them, TSMM reads A and
    # writes B.  (Prefix views of one wide buffer instead made some TSMM widths
    # up to 25% slower for reasons outside the kernels.)
    bufs = {}
    for cplx in (False, True):
        for i, (M, N) in enumerate(WIDTHS):
            bufs[cplx, M, N] = (inputs.device_uniform(K, M, i, inputs.STREAM_A, cplx, dev),
                                inputs.device_uniform(K, N, i, inputs.STREAM_B, cplx, dev))
    smallC = {c: inputs.device_uniform(64, 64, 0, inputs.STREAM_C, c, dev) for c in (False, True)}
    # Call order: per dtype all TSMTTSM widths, then all TSMM widths, each in
    # FLUSH_ORDER (a wide call between any two narrow ones), so that no call
    # finds the data of the call before it in the 256 MB Infinity Cache.
    calls = []
    for cplx in (False, True):
        for op in ("tsmttsm", "tsmm"):
            for (M, N) in FLUSH_ORDER:
                Av, Bv = bufs[cplx, M, N]
                if op == "tsmttsm":
                    Cout = torch.empty((M, N), dtype=Av.dtype, device=dev)
                    fn = (lambda Av=Av, Bv=Bv, Cout=Cout: api.tsmttsm(Av, Bv, out=Cout))
                else:
                    Cin = smallC[cplx][:M, :N].contiguous()
                    fn = (lambda Av=Av, Cin=Cin, Bv=Bv: api.tsmm(Av, Cin, out=Bv))
                calls.append(dict(op=op, cplx=cplx, M=M, N=N, fn=fn))
    for c in calls:
        c["bytes"], c["flops"] = algorithmic(c["op"], c["cplx"], K, c["M"], c["N"])
        c["kernel"] = api.kernel_name(c["op"], torch.complex128 if c["cplx"] else torch.float64, c["M"], c["N"])
    step_bytes = sum(c["bytes"] for c in calls)

    def step(events=None):
        for i, c in enumerate(calls):
            if events is not None:
                events[i][0].record()
            c["fn"]()
            if events is not None:
                events[i][1].record()

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    bs = measure_bs(torch, *bufs[True, 64, 64])   # 16 GiB each
    print("[bench] warmup done; b_s read %.0f GB/s, copy %.0f GB/s; timing %d steps"
          % (bs["read"] / 1e9, bs["copy"] / 1e9, a.steps), file=sys.stderr, flush=True)
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in calls]
           for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    per = []
    for i, c in enumerate(calls):
        ms = sum(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(a.steps)) / a.steps
        t = ms * 1e-3
        rt = roofline_time(c["bytes"], c["flops"])
        rt_bs = roofline_time(c["bytes"], c["flops"], bw=bs["read"] if c["op"] == "tsmttsm" else bs["copy"])
        per.append(dict(op=c["op"], dtype="Z" if c["cplx"] else "D", M=c["M"], N=c["N"], kernel=c["kernel"],
                        us=round(ms * 1e3, 2), GBps=round(c["bytes"] / t / 1e9, 1),
                        GFLOPs=round(c["flops"] / t / 1e9, 1), roof_frac=round(rt / t, 4),
                        roof_frac_bs=round(rt_bs / t, 4),
                        bound="fp64" if c["flops"] / FP64_PEAK > c["bytes"] / HBM_PEAK else "hbm"))
    dom_i = max(range(len(per)), key=lambda i: per[i]["us"])
    d = per[dom_i]
    dc = calls[dom_i]
    dt = d["us"] * 1e-6
    if d["bound"] == "hbm":
        roof = {"bound": "hbm", "achieved": round(dc["bytes"] / dt / 1e9, 1), "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": round(dc["bytes"] / dt / HBM_PEAK, 4)}
    else:
        roof = {"bound": "mfma", "achieved": round(dc["flops"] / dt / 1e12, 2), "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": round(dc["flops"] / dt / FP64_PEAK, 4)}
    from paper_1905_03136_amd import codegen, profile_summary
    src_hash = profile_summary.source_hash()
    symbol = codegen.kernel_symbol(d["kernel"])
    roof.update({"kernel": d["kernel"], "kernel_symbol": symbol, "avg_us": d["us"], "bytes": dc["bytes"],
                 "flops": dc["flops"], "traffic": None,
                 "per_launch": "%s %s M=%d N=%d K=%d: %d algorithmic bytes, %d flops" % (
                     d["op"], d["dtype"], d["M"], d["N"], K, dc["bytes"], dc["flops"])})
    # HBM bytes per launch from the committed counter summary of this step alone
    # (same kernel code), if there is one.  Only that summary qualifies: the
    # whole-bench summary averages kernels that the precision form also runs
    # at K = 2^25, so its per-launch bytes are not those of a K = 2^24 launch.
    f = os.path.join(ROOT, "profiles", "sweep_k2p24.md")
    rec = profile_summary.traffic_record(f, symbol, src_hash)
    if rec:
        roof["traffic"] = rec["traffic"]
        roof["traffic_source"] = "profiles/" + os.path.basename(f)

    if not a.no_check:
        # spot check of the timed buffers: one TSMTTSM entry against a direct FP64 dot product
        Av, Bv = bufs[False, 8, 8]
        C = api.tsmttsm(Av, Bv)
        ref = torch.dot(Av[:, 3].contiguous(), Bv[:, 5].contiguous())
        assert abs(float(C[3, 5] - ref)) <= 1e-10 * float(torch.dot(Av[:, 3].abs(), Bv[:, 5].abs()))

    out = {
        "metric": METRIC, "value": round(step_bytes * a.steps / (t1 - t0) / 1e9, 1), "unit": "GB/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "source_hash": src_hash,
        "data": "synthetic (seeded uniform(-1,1), generated on the device)",
        "config": {"workload": "plain width sweep: TSMTTSM and TSMM, D and Z, K=2^24, "
                               "(M,N) in {(1,1),(2,2),(4,4),(8,8),(16,16),(32,32),(64,64),(32,8),(8,32)}",
                   "calls_per_step": len(calls), "K": K, "bytes_per_step": step_bytes},
        "roofline": roof,
        "b_s": {"read_GBps": round(bs["read"] / 1e9, 1), "copy_GBps": round(bs["copy"] / 1e9, 1),
                "note": "measured with the library's stream probes over 8 GiB; roof_frac_bs uses b_s "
                        "(read for TSMTTSM, copy for TSMM) instead of the 8 TB/s spec"},
        "widths": per,
    }
    if not a.no_forms:
        del bufs, calls
        torch.cuda.empty_cache()
        print("[bench] precision form (binary32 storage) at K=2^25", file=sys.stderr, flush=True)
        out["precision_form"] = precision_form(torch, api, inputs, dev)
        torch.cuda.empty_cache()
        print("[bench] batched form (64 orthogonalisation steps, one persistent launch)", file=sys.stderr,
              flush=True)
        out["batched_form"] = batched_form(torch, api, inputs, dev)
    if a.cpu_sample > 0:
        print("[bench] timing the CPU oracle on a %d-row sample" % a.cpu_sample, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
