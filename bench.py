"""Throughput of the tall & skinny products on one MI355X.

One step is one pass of the plain width sweep: TSMTTSM (C = A^T B) and TSMM
(B = A C) in real (D) and complex (Z) double precision, K = 2^24 rows,
(M, N) in {(1,1), (2,2), (4,4), (8,8), (16,16), (32,32), (64,64), (32,8), (8,32)}:
36 calls on inputs already resident in HBM (seeded uniform(-1, 1) data,
generated on the device).  The value is the sweep's algorithmic bytes per
second (Eq. 1 of the paper: every element of A, B and C moves once); the JSON
line also carries each call's median / min / max time over the timed steps,
GB/s, GFLOP/s and fraction of the min(HBM, FP64) roofline, the roofline
record of the dominant kernel, the measured FP64 rates of the chip, clocks
and power, and the CPU oracle timed on the same sweep.  After the timed
steps (unless --no-forms) come the production forms and the other workload
sizes: the precision form (binary32 storage, binary64 and binary32
arithmetic, K = 2^25, with errors per result), the batched
orthogonalisation, the small-K product (K = 2^20, M = N = 4) and the
autograd form (K = 2^22, M = N = 32).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --all-widths      # every square width 1..64 instead (one JSON line each)
    python bench.py --all-widths --vendor   # ... with torch.matmul (rocBLAS / hipBLASLt) beside each
    python bench.py --reduction-sweep       # TSMTTSM reduction variants against K (ablation)
    python bench.py --pair-sweep            # nonsymmetric (M, N) grid
"""
import argparse
import json
import math
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


def time_stats(torch, fn, reps=5, warmup=1):
    """Median, minimum and maximum device time (s) of fn() over `reps` runs
    (events on the current stream)."""
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
    ts.sort()
    return {"median": ts[len(ts) // 2], "min": ts[0], "max": ts[-1]}


def time_call(torch, fn, reps=3, warmup=1):
    """Median device time of fn() over `reps` runs (events on the current stream)."""
    return time_stats(torch, fn, reps, warmup)["median"]


def time_steady(torch, fn, reps=3, warmup=1, span=1e-3):
    """Per-call device time of fn() in steady state: calls shorter than `span`
    are timed as a run of back-to-back calls lasting about `span` between one
    event pair (median of `reps` runs), so the host's time to issue each call
    overlaps the device's work as in a caller's loop; longer calls one by
    one."""
    t1 = time_stats(torch, fn, 1, warmup)["median"]
    n = 1 if t1 >= span else int(math.ceil(span / t1))
    if n == 1:
        return time_stats(torch, fn, reps, 0)["median"]

    def run():
        for _ in range(n):
            fn()
    return time_stats(torch, run, reps, 0)["median"] / n


def _host(t):
    """Device tensor -> numpy array in extended precision (values exact)."""
    import numpy as np
    x = t.detach().cpu().numpy()
    return x.astype(np.clongdouble if np.iscomplexobj(x) else np.longdouble)


def _exact_entries(torch, A, B, entries, conj=False):
    """Entries (m, n) of op(A)^T B from the stored values, computed on the
    host: every product of two values is formed and summed in 80-bit extended
    precision (products of binary32 values are exact there; a pairwise sum of
    K <= 2^25 terms errs by at most about 25 * 2^-64 relative to sum |a b|),
    i.e. a reference far more accurate than either arithmetic it judges.
    Returns (values, sum |a| |b|) per entry."""
    import numpy as np
    cols = {}
    vals, absb = [], []
    for m, n in entries:
        if ("a", m) not in cols:
            cols["a", m] = _host(A[:, m])
        if ("b", n) not in cols:
            cols["b", n] = _host(B[:, n])
        a, b = cols["a", m], cols["b", n]
        if conj:
            a = np.conj(a)
        vals.append(np.sum(a * b))
        absb.append(np.sum(np.abs(a) * np.abs(b)))
    return np.array(vals), np.array(absb)


def _exact_rows(torch, A, C, rows):
    """Rows of A C from the stored values, in extended precision (see
    _exact_entries); returns (rows of A C, rows of |A| |C|)."""
    import numpy as np
    idx = torch.as_tensor(rows, device=A.device)
    a = _host(A.index_select(0, idx))
    c = _host(C)
    return (a[:, :, None] * c[None, :, :]).sum(axis=1), (np.abs(a)[:, :, None] * np.abs(c)[None, :, :]).sum(axis=1)


def _errors(got, ref, absb):
    """Normwise and elementwise relative errors and the cancellation-free
    measure max |got - ref| / (|a|^T |b|) over the sampled entries."""
    import numpy as np
    got = np.asarray(got).astype(ref.dtype)
    d = np.abs(got - ref)
    return {"normwise": float(np.sqrt(np.sum(d ** 2)) / np.sqrt(np.sum(np.abs(ref) ** 2))),
            "max_elementwise": float(np.max(d / np.maximum(np.abs(ref), 1e-300))),
            "max_vs_abs_products": float(np.max(d / np.maximum(absb, 1e-300)))}


# the storage / arithmetic forms of the precision bench: (name, storage, arithmetic)
PREC_FORMS = [("fp64", "binary64", "binary64"), ("fp32_acc64", "binary32", "binary64"),
              ("fp32_acc32", "binary32", "binary32")]


def precision_form(torch, api, inputs, dev, K=1 << 25, widths=(8, 32, 64), nrows=64):
    """The precision form against binary64 storage at K = 2^25, real and
    complex, M = N in `widths`, both products: binary32 / complex64 storage
    of the tall operands with binary64 arithmetic (values widened exactly,
    products exact, binary64 sums) and with binary32 arithmetic (binary32
    products on the matrix cores summed in binary32 over 32-row stretches,
    binary64 beyond and across blocks).  Per result: time, speedup over
    binary64 storage, and the error on sampled outputs (TSMTTSM: entries
    (0, 0), (w-1, w/2), (w/2, w-1); TSMM: `nrows` rows spread over K) against
    the exact result of the stored values ("arithmetic") and of the binary64
    data before storage rounding ("end to end"), for uniform(-1, 1) data and
    for the ill-conditioned case: near-parallel columns base + 1e-4 noise_j,
    TSMTTSM as the Gram matrix A^T A, TSMM with a small matrix whose columns
    sum to zero (so that A C cancels by about 1e4)."""
    import numpy as np
    out = []
    for cplx in (False, True):
        t64 = torch.complex128 if cplx else torch.float64
        t32 = torch.complex64 if cplx else torch.float32
        sz = 16 if cplx else 8
        for w in widths:
            rec = {"dtype": "Z" if cplx else "D", "M": w, "N": w, "K": K}
            entries = sorted({(0, 0), (w - 1, w // 2), (w // 2, w - 1)})
            rows = [int(r) for r in np.linspace(0, K - 1, nrows).round()]
            for case in ("uniform", "ill_conditioned"):
                if case == "uniform":
                    A = inputs.device_uniform(K, w, 7 + w, inputs.STREAM_A, cplx, dev)
                    B = inputs.device_uniform(K, w, 7 + w, inputs.STREAM_B, cplx, dev)
                    X = inputs.device_uniform(w, w, 7 + w, inputs.STREAM_C, cplx, dev)
                else:
                    base = inputs.device_uniform(K, 1, 7 + w, inputs.STREAM_BASE, cplx, dev)
                    A = inputs.device_uniform(K, w, 7 + w, inputs.STREAM_NOISE0, cplx, dev)
                    A.mul_(1e-4).add_(base)
                    del base
                    B = A
                    X = torch.from_numpy(inputs.zero_column_sum(w, w, 7 + w, inputs.STREAM_C, cplx)).to(dev)
                A32 = A.to(t32)
                B32 = A32 if B is A else B.to(t32)
                Bout = torch.empty((K, w), dtype=t64, device=dev)
                Bout32 = torch.empty((K, w), dtype=t32, device=dev)
                # exact references: of the stored binary32 values, and of the binary64 data
                ref32, ab32 = _exact_entries(torch, A32, B32, entries)
                ref64, ab64 = _exact_entries(torch, A, B, entries)
                rref32, rab32 = _exact_rows(torch, A32, X, rows)
                rref64, rab64 = _exact_rows(torch, A, X, rows)
                res = {}
                for op in ("tsmttsm", "tsmm"):
                    r = {}
                    for name, storage, arith in PREC_FORMS:
                        a, b = (A, B) if storage == "binary64" else (A32, B32)
                        acc = "f32" if arith == "binary32" else "f64"
                        if op == "tsmttsm":
                            Cout = torch.empty((w, w), dtype=t64, device=dev)
                            fn = (lambda a=a, b=b, acc=acc, Cout=Cout: api.tsmttsm(a, b, out=Cout, acc=acc))
                        else:
                            o = Bout if storage == "binary64" else Bout32
                            fn = (lambda a=a, acc=acc, o=o: api.tsmm(a, X, out=o, acc=acc))
                        st = time_stats(torch, fn, reps=5, warmup=1) if case == "uniform" else None
                        fn()
                        torch.cuda.synchronize()
                        if op == "tsmttsm":
                            got = np.array([Cout[m, n].item() for m, n in entries])
                            e_ar = _errors(got, ref32 if storage == "binary32" else ref64,
                                           ab32 if storage == "binary32" else ab64)
                            e_ee = _errors(got, ref64, ab64)
                        else:
                            o = Bout if storage == "binary64" else Bout32
                            got = o.index_select(0, torch.as_tensor(rows, device=dev)).cpu().numpy()
                            e_ar = _errors(got, rref32 if storage == "binary32" else rref64,
                                           rab32 if storage == "binary32" else rab64)
                            e_ee = _errors(got, rref64, rab64)
                        item = {"error_arithmetic": e_ar, "error_end_to_end": e_ee,
                                "kernel": api.kernel_name(op, t64 if storage == "binary64" else t32, w, w, acc=acc)}
                        if st:
                            byts = (sz if storage == "binary64" else sz // 2) * K * 2 * w + sz * w * w
                            item.update(us=round(st["median"] * 1e6, 1), us_min=round(st["min"] * 1e6, 1),
                                        us_max=round(st["max"] * 1e6, 1), GBps=round(byts / st["median"] / 1e9, 1))
                        r[name] = item
                    if case == "uniform":
                        for name, _, _ in PREC_FORMS[1:]:
                            r[name]["speedup_vs_fp64"] = round(r["fp64"]["us"] / r[name]["us"], 3)
                    res[op] = r
                rec[case] = res
                del A, B, A32, B32, Bout, Bout32, X
                torch.cuda.empty_cache()
            out.append(rec)
            print("[bench] precision form %s %dx%d: speedup TSMTTSM %.2f / %.2f, TSMM %.2f / %.2f "
                  "(binary64 / binary32 arithmetic)" % (
                      rec["dtype"], w, w, rec["uniform"]["tsmttsm"]["fp32_acc64"]["speedup_vs_fp64"],
                      rec["uniform"]["tsmttsm"]["fp32_acc32"]["speedup_vs_fp64"],
                      rec["uniform"]["tsmm"]["fp32_acc64"]["speedup_vs_fp64"],
                      rec["uniform"]["tsmm"]["fp32_acc32"]["speedup_vs_fp64"]), file=sys.stderr, flush=True)
    return {"note": "fp64: binary64 / complex128 storage; fp32_acc64: binary32 / complex64 storage, values "
                    "widened exactly, binary64 products and sums; fp32_acc32: binary32 storage, binary32 "
                    "products summed in binary32 over 32-row stretches (TSMM: over the M terms of one "
                    "output), binary64 beyond and across blocks.  error_arithmetic is against the exact result "
                    "of the stored values, error_end_to_end against the exact result of the binary64 data "
                    "before it was rounded to binary32 (both formed on the host in 80-bit extended "
                    "precision), on sampled outputs: TSMTTSM entries (0,0), (w-1,w/2), (w/2,w-1); TSMM 64 "
                    "rows spread over K.  ill_conditioned: columns base + 1e-4 noise_j; TSMTTSM computes the "
                    "Gram matrix A^T A, TSMM multiplies by a small matrix with zero column sums",
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
    # the same step through tsg_orth_batched (descriptors in device memory,
    # the queue built on the device by a set-up kernel, then the same
    # persistent kernel), direct and captured in a graph
    ob = api.OrthBatch(pairs)
    t_batched = time_call(torch, ob.run, reps=reps, warmup=2)
    ob.check()
    sb = torch.cuda.Stream()
    sb.wait_stream(torch.cuda.current_stream())
    gb = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gb, stream=sb):
        ob.run()
    t_batched_graph = time_call(torch, gb.replay, reps=reps, warmup=2)
    ob.check()
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
    del g, gb, ob
    return {"instances": 64, "rows": sum(k for k, _, _ in shapes),
            "algorithmic_bytes": byts, "cache_ideal_bytes": ideal, "flops": flops,
            "us_persistent_graph": round(t_persist * 1e6, 1), "us_128_launches": round(t_sep * 1e6, 1),
            "us_orth_batched": round(t_batched * 1e6, 1), "us_orth_batched_graph": round(t_batched_graph * 1e6, 1),
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


def small_k_leg(torch, api, inputs, dev, K=1 << 20, M=4, N=4, sets=20, reps=5):
    """TSMTTSM, real, K = 2^20 rows, M = N = 4 (67 MB per call, inside the
    256 MB Infinity Cache): `sets` distinct operand pairs (1.3 GB in all) are
    used in turn so that no call finds its operands in the cache, as a
    caller's stream of independent small products would.  Median, minimum
    and maximum per-call time over reps passes over the sets."""
    pairs = [(inputs.device_uniform(K, M, 50 + i, inputs.STREAM_A, False, dev),
              inputs.device_uniform(K, N, 50 + i, inputs.STREAM_B, False, dev)) for i in range(sets)]
    C = torch.empty((M, N), dtype=torch.float64, device=dev)
    for a, b in pairs:
        api.tsmttsm(a, b, out=C)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        evs = []
        for a, b in pairs:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            api.tsmttsm(a, b, out=C)
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ts += [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
    ts.sort()
    t = ts[len(ts) // 2]
    byts, flops = algorithmic("tsmttsm", False, K, M, N)
    # The same calls captured in one hipGraph and replayed (a launch-bound
    # loop's deployment): per-call device time without the host's time to
    # issue each call, which the eager figure above includes whenever the
    # host is slower than the kernels.  Each replay is checked against the
    # eager results.
    cs = torch.cuda.Stream()
    Cs = [torch.empty((M, N), dtype=torch.float64, device=dev) for _ in pairs]
    with torch.cuda.stream(cs):
        for (a, b), c in zip(pairs, Cs):
            api.tsmttsm(a, b, out=c)      # sizes the capture stream's workspace
    cs.synchronize()
    eager = [c.clone() for c in Cs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        for (a, b), c in zip(pairs, Cs):
            api.tsmttsm(a, b, out=c)
    tg = []
    for _ in range(reps):
        for c in Cs:
            c.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        tg.append(e0.elapsed_time(e1) * 1e-3 / len(pairs))
        assert all(torch.equal(c, e) for c, e in zip(Cs, eager)), "graph replay differs from the eager calls"
    tg.sort()
    t_graph = tg[len(tg) // 2]
    del pairs, g
    return {"workload": "TSMTTSM D K=2^20 M=N=4, %d operand sets rotated (%.2f GB)" % (sets, sets * 8 * K * (M + N) / 1e9),
            "us": round(t * 1e6, 2), "us_min": round(ts[0] * 1e6, 2), "us_max": round(ts[-1] * 1e6, 2),
            "GBps": round(byts / t / 1e9, 1), "roof_frac": round(roofline_time(byts, flops) / t, 4),
            "us_graph": round(t_graph * 1e6, 2), "GBps_graph": round(byts / t_graph / 1e9, 1),
            "roof_frac_graph": round(roofline_time(byts, flops) / t_graph, 4),
            "kernel": api.kernel_name("tsmttsm", torch.float64, M, N), "calls_timed": len(ts),
            "note": "us: eager calls, one event pair each (includes the host's issue time when it exceeds the "
                    "kernel's); us_graph: the %d calls replayed from one captured graph, per call" % len(Cs)}


def autograd_leg(torch, inputs, dev, K=1 << 22, w=32, reps=5):
    """The differentiation form at K = 2^22, M = N = 32, real and complex:
    forward C = A^T B through autograd.TSMTTSM, backward dA = B dC^T,
    dB = A dC (complex: the conjugate forms) on the TSMM kernels, dC uniform.
    Algorithmic bytes: forward s K (M + N) + s M N; backward two TSMMs,
    2 s K (M + N) + 2 s M N."""
    from paper_1905_03136_amd import autograd
    out = []
    for cplx in (False, True):
        A = inputs.device_uniform(K, w, 9, inputs.STREAM_A, cplx, dev).requires_grad_(True)
        B = inputs.device_uniform(K, w, 9, inputs.STREAM_B, cplx, dev).requires_grad_(True)
        dC = inputs.device_uniform(w, w, 9, inputs.STREAM_DC, cplx, dev)
        holder = {}

        def fwd():
            holder["C"] = autograd.tsmttsm(A, B)

        def bwd():
            A.grad = B.grad = None
            holder["C"].backward(dC, retain_graph=True)

        tf = time_stats(torch, fwd, reps=reps, warmup=1)
        fwd()
        tb = time_stats(torch, bwd, reps=reps, warmup=1)
        # back to back (as a training loop issues them): per-call time of 8
        # calls between one event pair, the host's issue time overlapped
        tfp = time_stats(torch, lambda: [fwd() for _ in range(8)], reps=3, warmup=1)["median"] / 8
        fwd()
        tbp = time_stats(torch, lambda: [bwd() for _ in range(8)], reps=3, warmup=1)["median"] / 8
        s = 16 if cplx else 8
        fb = s * K * 2 * w + s * w * w
        bb = 2 * s * K * 2 * w + 2 * s * w * w
        ff = (8 if cplx else 2) * w * w * K
        out.append({"dtype": "Z" if cplx else "D", "K": K, "M": w, "N": w,
                    "forward_us": round(tf["median"] * 1e6, 1), "backward_us": round(tb["median"] * 1e6, 1),
                    "forward_GBps": round(fb / tf["median"] / 1e9, 1), "backward_GBps": round(bb / tb["median"] / 1e9, 1),
                    "forward_roof_frac": round(roofline_time(fb, ff) / tf["median"], 4),
                    "backward_roof_frac": round(roofline_time(bb, 2 * ff) / tb["median"], 4),
                    "forward_us_back_to_back": round(tfp * 1e6, 1), "backward_us_back_to_back": round(tbp * 1e6, 1),
                    "forward_roof_frac_back_to_back": round(roofline_time(fb, ff) / tfp, 4),
                    "backward_roof_frac_back_to_back": round(roofline_time(bb, 2 * ff) / tbp, 4)})
        del A, B, dC, holder
        torch.cuda.empty_cache()
    return out


def fp64_peaks(torch, occs=(1, 2, 4, 8), iters=20000):
    """Measured FP64 rates of the chip (the paper computes its own peak,
    Section 1.6): register-only loops of the library's peak probes with eight
    independent matrix-core (or sixteen vector FMA) chains per lane, the best
    over blocks of 256 threads per CU; and the binary32 matrix-core rate."""
    from paper_1905_03136_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    kinds = {"mfma_f64": _lib.TSG_PEAK_MFMA_F64, "valu_f64": _lib.TSG_PEAK_VALU_F64,
             "mixed_f64": _lib.TSG_PEAK_MIXED_F64, "mfma_f32": _lib.TSG_PEAK_MFMA_F32}
    out = {}
    for name, kind in kinds.items():
        per = {}
        for occ in occs:
            fl = [0.0]

            def run():
                st, fl[0] = _lib.tsg_peak_probe(kind, occ, iters, s)
                _lib.check(st)
            t = time_call(torch, run, reps=3)   # runs the probe, which sets fl[0]
            per[str(occ)] = round(fl[0] / t / 1e12, 2)
        out[name] = {"TFLOPs_by_blocks_per_cu": per, "best_TFLOPs": max(per.values())}
    return out


def gpu_state():
    """Clocks and power as rocm-smi reports them (None where it is missing)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--json"], stdout=subprocess.PIPE,
                           stderr=subprocess.DEVNULL, text=True, timeout=30)
        d = json.loads(r.stdout)
        card = d[sorted(d)[0]]
        keep = {k: v for k, v in card.items() if "clk" in k.lower() or "power" in k.lower()}
        return keep or None
    except Exception:
        return None


def cpu_baseline(K_sample):
    """The oracle as it stands, timed on the host over the bench step's 36
    calls at K_sample rows.  It splits the independent output rows over its
    threads (rows of C for TSMTTSM: at most M threads; rows of B for TSMM:
    all of them), so `cores` is the time-weighted mean of the threads the
    calls actually kept busy; the per-call counts are listed too."""
    import numpy as np

    import oracle
    from paper_1905_03136_amd import inputs
    oracle.build()
    threads = oracle.max_threads()
    total_bytes = 0
    t_total = 0.0
    busy = 0.0
    per = []
    for cplx in (False, True):
        A = inputs.host_uniform(K_sample, 64, 0, inputs.STREAM_A, cplx)
        B = inputs.host_uniform(K_sample, 64, 0, inputs.STREAM_B, cplx)
        Xfull = inputs.host_uniform(64, 64, 0, inputs.STREAM_C, cplx)
        for (M, N) in WIDTHS:
            a = np.ascontiguousarray(A[:, :M])
            b = np.ascontiguousarray(B[:, :N])
            X = np.ascontiguousarray(Xfull[:M, :N])
            for op in ("tsmttsm", "tsmm"):
                t0 = time.perf_counter()
                if op == "tsmttsm":
                    oracle.tsmttsm(a, b)
                else:
                    oracle.tsmm(a, X)
                dt = time.perf_counter() - t0
                used = min(M, threads) if op == "tsmttsm" else threads
                t_total += dt
                busy += used * dt
                total_bytes += algorithmic(op, cplx, K_sample, M, N)[0]
                per.append({"op": op, "dtype": "Z" if cplx else "D", "M": M, "N": N, "s": round(dt, 3),
                            "threads": used})
            del a, b
        del A, B
    return {"value": total_bytes / t_total / 1e9, "unit": "GB/s", "cores": round(busy / t_total, 2),
            "kind": "oracle",
            "sample": "the bench step's 36 calls (TSMTTSM+TSMM, D and Z, 9 widths) at K=%d rows; plain "
                      "binary64 triple loop, threads over output rows; %.1f s" % (K_sample, t_total),
            "host_threads": threads, "seconds": t_total, "calls": per,
            "cpu": platform.processor() or platform.machine(), "nproc": os.cpu_count()}


def all_widths(torch, api, inputs, dev, K=K_SWEEP, reps=3, vendor=False, widths=tuple(range(1, 65))):
    """Every square width M = N = 1..64, D and Z, both products at K rows:
    steady-state time per call (median of `reps`; calls under 1 ms as a run
    of back-to-back calls, see time_steady; one width at a time, exact-size
    operands)
    and the fraction of the spec roofline; one JSON line per width, then a
    summary line with the mean and the minimum fraction per (dtype, op).
    With `vendor`, the same products through torch.matmul (rocBLAS /
    hipBLASLt GEMMs: A^T B as a transposed view times B, A C) are timed on
    the same operands beside ours -- the vendor-library context of the
    paper's library comparison (Section 1.5), measured on this GPU."""
    rows = []
    for cplx in (False, True):
        for w in widths:
            A = inputs.device_uniform(K, w, w, inputs.STREAM_A, cplx, dev)
            B = inputs.device_uniform(K, w, w, inputs.STREAM_B, cplx, dev)
            X = inputs.device_uniform(w, w, w, inputs.STREAM_C, cplx, dev)
            Co = torch.empty((w, w), dtype=A.dtype, device=dev)
            rec = {"dtype": "Z" if cplx else "D", "M": w, "N": w, "K": K}
            for op, fn in (("tsmttsm", lambda: api.tsmttsm(A, B, out=Co)), ("tsmm", lambda: api.tsmm(A, X, out=B))):
                t = time_steady(torch, fn, reps=reps, warmup=1)
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


def pair_sweep(torch, api, inputs, dev, widths=(1, 4, 8, 16, 24, 32, 40, 48, 56, 64), K=K_SWEEP, reps=3):
    """Nonsymmetric widths: every (M, N) with M and N in `widths`, D and Z, both
    products at K rows (the paper measures only M = N and calls the other
    shapes "not fundamentally different", Section 1.3).  One JSON line per
    pair, then a summary with the mean and minimum fraction of the spec
    roofline per (dtype, operation) and how many pairs reach 0.8."""
    rows = []
    for cplx in (False, True):
        for M in widths:
            for N in widths:
                A = inputs.device_uniform(K, M, M, inputs.STREAM_A, cplx, dev)
                B = inputs.device_uniform(K, N, N, inputs.STREAM_B, cplx, dev)
                X = inputs.device_uniform(M, N, M + N, inputs.STREAM_C, cplx, dev)
                Co = torch.empty((M, N), dtype=A.dtype, device=dev)
                rec = {"dtype": "Z" if cplx else "D", "M": M, "N": N, "K": K}
                for op, fn in (("tsmttsm", lambda: api.tsmttsm(A, B, out=Co)), ("tsmm", lambda: api.tsmm(A, X, out=B))):
                    t = time_steady(torch, fn, reps=reps, warmup=1)
                    byts, flops = algorithmic(op, cplx, K, M, N)
                    rec[op] = {"us": round(t * 1e6, 1), "roof_frac": round(roofline_time(byts, flops) / t, 4),
                               "kernel": api.kernel_name(op, A.dtype, M, N)}
                print(json.dumps(rec), flush=True)
                rows.append(rec)
                del A, B, X, Co
    summary = {}
    for dt in ("D", "Z"):
        for op in ("tsmttsm", "tsmm"):
            f = [r[op]["roof_frac"] for r in rows if r["dtype"] == dt]
            summary["%s_%s" % (dt, op)] = {"mean": round(sum(f) / len(f), 4), "min": min(f),
                                           "pairs": len(f), "at_least_0.8": sum(1 for x in f if x >= 0.8)}
    print(json.dumps({"pair_sweep_summary": summary}), flush=True)


def pair_table(path):
    """Markdown tables (fraction of the roofline, rows M, columns N) of the
    JSON lines a --pair-sweep run printed, one table per dtype and product,
    followed by the summary line."""
    rows, summary = [], None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line.startswith("{"):
                continue
            r = json.loads(line)
            if "pair_sweep_summary" in r:
                summary = r
            else:
                rows.append(r)
    Ms = sorted({r["M"] for r in rows})
    Ns = sorted({r["N"] for r in rows})
    out = []
    for dt in ("D", "Z"):
        for op in ("tsmttsm", "tsmm"):
            cell = {(r["M"], r["N"]): r[op]["roof_frac"] for r in rows if r["dtype"] == dt}
            out.append("**%s %s** (rows M, columns N)\n" % (dt, op.upper()))
            out.append("| M \\\\ N | " + " | ".join(str(n) for n in Ns) + " |")
            out.append("|---|" + "---:|" * len(Ns))
            for m in Ms:
                out.append("| %d | " % m + " | ".join("%.2f" % cell[m, n] if (m, n) in cell else "" for n in Ns)
                           + " |")
            out.append("")
    if summary:
        out.append("```json\n%s\n```" % json.dumps(summary, indent=1))
    return "\n".join(out)


def vendor_table(path):
    """Markdown table of the JSON lines an --all-widths --vendor run printed."""
    rows, summary = [], None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line.startswith("{"):
                continue
            r = json.loads(line)
            if "all_widths_summary" in r:
                summary = r
            elif "vendor_us" in r.get("tsmttsm", {}):
                rows.append(r)
    out = ["| dtype | w | TSMTTSM ours us | vendor us | ours / vendor speedup | TSMM ours us | vendor us | speedup "
           "| ours frac (T / M) | vendor frac (T / M) |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---|---|"]
    for r in rows:
        t, m = r["tsmttsm"], r["tsmm"]
        out.append("| %s | %d | %.1f | %.1f | %.0f | %.1f | %.1f | %.2f | %.3f / %.3f | %.4f / %.3f |" % (
            r["dtype"], r["M"], t["us"], t["vendor_us"], t["speedup_vs_vendor"], m["us"], m["vendor_us"],
            m["speedup_vs_vendor"], t["roof_frac"], m["roof_frac"], t["vendor_roof_frac"], m["vendor_roof_frac"]))
    if summary:
        out.append("\nSummary over these widths:\n\n```json\n%s\n```" % json.dumps(summary, indent=1))
    return "\n".join(out)


def reduction_table(path):
    """Markdown table of the JSON lines a --reduction-sweep run printed."""
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                r = json.loads(line)
                if "fold" in r:
                    rows.append(r)
    out = ["| M = N | K | fold us | fold overhead | atomic us | atomic overhead | none us | fraction (fold) |",
           "|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %d | %d | %.1f | %+.0f%% | %.1f | %+.0f%% | %.1f | %.3f |" % (
            r["M"], r["K"], r["fold"]["us"], 100 * r["fold"]["overhead_vs_none"], r["atomic"]["us"],
            100 * r["atomic"]["overhead_vs_none"], r["none"]["us"], r["fold"]["roof_frac"]))
    out.append("\n```json\n%s\n```" % json.dumps(rows))
    return "\n".join(out)


def reduction_sweep(torch, api, inputs, dev, widths=(4, 32), Ks=(10**3, 10**4, 10**5, 10**6, 10**7, 10**8),
                    reps=20):
    """Ablation of TSMTTSM's cross-block reduction against K (the paper's
    Sections 3.2 and 5.5): the fixed-order two-kernel fold (the library's
    default), global FP64 atomics of every block's partial into C, and no
    reduction at all (the kernel alone: a lower bound), real data, M = N in
    `widths`.  Per K up to 64 operand sets of at least 1 GiB together are used
    in turn where they fit (small K stays cache resident, as in the paper's
    sweep); median of `reps` event-timed calls.  One JSON line per (width, K)."""
    from paper_1905_03136_amd import _lib
    modes = (("fold", _lib.TSG_REDUCE_FOLD), ("atomic", _lib.TSG_REDUCE_ATOMIC), ("none", _lib.TSG_REDUCE_NONE))
    for w in widths:
        for K in Ks:
            per = 8 * K * 2 * w
            sets = max(1, min(64, -(-(1 << 30) // per)))
            pairs = [(inputs.device_uniform(K, w, 60 + i, inputs.STREAM_A, False, dev),
                      inputs.device_uniform(K, w, 60 + i, inputs.STREAM_B, False, dev)) for i in range(sets)]
            C = torch.empty((w, w), dtype=torch.float64, device=dev)
            byts, flops = algorithmic("tsmttsm", False, K, w, w)
            rec = {"M": w, "N": w, "K": K, "sets": sets, "kernel": api.kernel_name("tsmttsm", torch.float64, w, w)}
            try:
                for name, mode in modes:
                    _lib.check(_lib.tsg_set_reduction(mode))
                    for a, b in pairs[:2]:
                        api.tsmttsm(a, b, out=C)
                    torch.cuda.synchronize()
                    ts = []
                    for r in range(reps):
                        a, b = pairs[r % sets]
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        api.tsmttsm(a, b, out=C)
                        e1.record()
                        e1.synchronize()
                        ts.append(e0.elapsed_time(e1) * 1e-3)
                    ts.sort()
                    t = ts[len(ts) // 2]
                    rec[name] = {"us": round(t * 1e6, 2), "GBps": round(byts / t / 1e9, 1),
                                 "roof_frac": round(roofline_time(byts, flops) / t, 4)}
            finally:
                _lib.tsg_set_reduction(_lib.TSG_REDUCE_FOLD)
            for name in ("fold", "atomic"):
                rec[name]["overhead_vs_none"] = round(rec[name]["us"] / rec["none"]["us"] - 1.0, 4)
            print(json.dumps(rec), flush=True)
            del pairs
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    # 2^24 rows, the bench's own K: the 36 calls move 268 GB, about 17 s of
    # oracle work on 16 host threads (15.4 GB/s measured at 2^23 rows);
    # host inputs of at most 17.2 GB per matrix
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="rows of the oracle sample (0 = skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the post-run spot check")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision / batched form measurements")
    ap.add_argument("--no-smi", action="store_true", help="do not query rocm-smi for clocks and power")
    ap.add_argument("--all-widths", action="store_true",
                    help="instead of the bench step: every square width 1..64 (D, Z, both products), one JSON line each")
    ap.add_argument("--width-list", default="", help="with --all-widths: comma-separated square widths (default 1..64)")
    ap.add_argument("--pair-sweep", action="store_true",
                    help="instead of the bench step: nonsymmetric (M, N) grid, D and Z, both products")
    ap.add_argument("--pair-table", default="",
                    help="no GPU: print the markdown tables of a --pair-sweep run's JSON lines (file) and exit")
    ap.add_argument("--vendor-table", default="",
                    help="no GPU: print the markdown table of an --all-widths --vendor run's JSON lines (file) and exit")
    ap.add_argument("--reduction-table", default="",
                    help="no GPU: print the markdown table of a --reduction-sweep run's JSON lines (file) and exit")
    ap.add_argument("--reduction-sweep", action="store_true",
                    help="instead of the bench step: TSMTTSM reduction variants (fold / atomic / none) against K")
    ap.add_argument("--vendor", action="store_true",
                    help="with --all-widths: also time torch.matmul (rocBLAS / hipBLASLt) on the same operands")
    a = ap.parse_args()
    if a.pair_table:
        print(pair_table(a.pair_table))
        return
    if a.reduction_table:
        print(reduction_table(a.reduction_table))
        return
    if a.vendor_table:
        print(vendor_table(a.vendor_table))
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the products run on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_03136_amd import api, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.all_widths:
        ws = tuple(int(x) for x in a.width_list.split(",")) if a.width_list else tuple(range(1, 65))
        all_widths(torch, api, inputs, dev, vendor=a.vendor, widths=ws)
        return
    if a.reduction_sweep:
        reduction_sweep(torch, api, inputs, dev)
        return
    if a.pair_sweep:
        pair_sweep(torch, api, inputs, dev)
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
    gpu_before = None if a.no_smi else gpu_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    gpu_after = None if a.no_smi else gpu_state()
    per = []
    for i, c in enumerate(calls):
        ts = sorted(evs[s][i][0].elapsed_time(evs[s][i][1]) * 1e-3 for s in range(a.steps))
        t = ts[len(ts) // 2]
        rt = roofline_time(c["bytes"], c["flops"])
        rt_bs = roofline_time(c["bytes"], c["flops"], bw=bs["read"] if c["op"] == "tsmttsm" else bs["copy"])
        per.append(dict(op=c["op"], dtype="Z" if c["cplx"] else "D", M=c["M"], N=c["N"], kernel=c["kernel"],
                        us=round(t * 1e6, 2), us_min=round(ts[0] * 1e6, 2), us_max=round(ts[-1] * 1e6, 2),
                        GBps=round(c["bytes"] / t / 1e9, 1),
                        GFLOPs=round(c["flops"] / t / 1e9, 1), roof_frac=round(rt / t, 4),
                        roof_frac_bs=round(rt_bs / t, 4),
                        bound="fp64" if c["flops"] / FP64_PEAK > c["bytes"] / HBM_PEAK else "hbm"))
    peaks = fp64_peaks(torch)
    dom_i = max(range(len(per)), key=lambda i: per[i]["us"])
    d = per[dom_i]
    dc = calls[dom_i]
    dt = d["us"] * 1e-6
    # a complex kernel in the three-product (Gauss) form executes 6MNK of the
    # 8MNK algorithmic flops on the matrix cores
    g3 = dc["cplx"] and "_g3" in d["kernel"]
    executed = dc["flops"] * 6 // 8 if g3 else dc["flops"]
    if d["bound"] == "hbm":
        roof = {"bound": "hbm", "achieved": round(dc["bytes"] / dt / 1e9, 1), "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": round(dc["bytes"] / dt / HBM_PEAK, 4)}
    else:
        roof = {"bound": "mfma", "achieved": round(dc["flops"] / dt / 1e12, 2), "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": round(dc["flops"] / dt / FP64_PEAK, 4),
                "executed_flops": executed, "executed_TFLOPs": round(executed / dt / 1e12, 2),
                "executed_frac": round(executed / dt / FP64_PEAK, 4),
                "peak_measured_mfma_f64": peaks["mfma_f64"]["best_TFLOPs"],
                "frac_of_measured_mfma_f64": round(executed / dt / 1e12 / peaks["mfma_f64"]["best_TFLOPs"], 4)}
    from paper_1905_03136_amd import codegen, profile_summary
    src_hash = profile_summary.source_hash()
    symbol = codegen.kernel_symbol(d["kernel"])
    roof.update({"kernel": d["kernel"], "kernel_symbol": symbol, "avg_us": d["us"], "bytes": dc["bytes"],
                 "flops": dc["flops"], "traffic": None, "timing": "median over the timed steps (HIP events on "
                 "the launch stream)",
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
        # the same fraction from the profiler's kernel trace of that run
        tt = rec["avg_us"] * 1e-6
        roof["trace_avg_us"] = rec["avg_us"]
        roof["frac_trace"] = round((dc["bytes"] / tt / HBM_PEAK) if d["bound"] == "hbm" else
                                   (dc["flops"] / tt / FP64_PEAK), 4)

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
        "fp64_peaks_measured": peaks,
        "gpu_state": {"before": gpu_before, "after": gpu_after},
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
        torch.cuda.empty_cache()
        print("[bench] small-K leg (TSMTTSM D K=2^20 M=N=4) and autograd leg (K=2^22, 32x32)", file=sys.stderr,
              flush=True)
        out["small_k"] = small_k_leg(torch, api, inputs, dev)
        out["autograd_form"] = autograd_leg(torch, inputs, dev)
    if a.cpu_sample > 0:
        print("[bench] timing the CPU oracle on a %d-row sample" % a.cpu_sample, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
