"""Performance model of the generated kernels, used to prune the autotuner.

The paper closes (Section 7) with a performance model as future work; its own
analysis (Sections 1.6 and 5.3) bounds a kernel by the memory bandwidth it can
reach with the loads it keeps in flight (Little's law over the latency of
Table 1's measurements) and by the arithmetic rate.  The model here does the
same with this chip's measured constants:

  t = max( bytes / BW(q),  FP64 matrix-core flops / P_mfma,  vector flops / P_valu ) + t_launch

* q, the bytes in flight per compute unit: blocks resident per CU (from the
  kernel's register and LDS use) x the bytes one block has requested ahead of
  its multiplications (the register sets of its leap-frog ring beyond the one
  being multiplied, or the LDS stage in flight);
* the matrix-core rate falls with one resident wave per SIMD (the peak probe
  keeps the FP64 matrix core busy 48% of the cycles with one wave, 66% with
  two or more);
* BW(q): the read bandwidth the Table-1 probe measured at that many bytes in
  flight per CU (interpolated; saturating at b_s), lowered for the read+write
  stream of TSMM to the measured ceiling of its read:write mix;
* P_mfma, P_valu: the measured FP64 matrix-core and vector rates (peak probes
  and the best kernel's executed rate from the instruction counters); complex
  kernels in the three-product form execute 6MNK instead of 8MNK flops.

It is deliberately coarse: it ranks configurations so that the tuner need not
time those predicted far slower than the best prediction (``prune``), and
``evaluate`` measures on a tuning database how often the measured fastest
configuration survives the pruning.

    python -m paper_1905_03136_amd.model evaluate --db DB.jsonl [--keep 1.3] [--tag tune]
"""
import argparse
import bisect
import collections
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# Measured on one MI355X (the probes of probes.py and the counters of the bench):
# read bandwidth (GB/s) against bytes in flight per CU (256-thread blocks x
# loads in flight x 16 B), Table-1 grid
TABLE1 = [(4 << 10, 2350.0), (8 << 10, 3950.0), (16 << 10, 6200.0), (32 << 10, 7100.0), (64 << 10, 7050.0),
          (256 << 10, 7000.0)]
MIX_CEILING = {(1, 1): 5384.0, (2, 1): 5836.0, (4, 1): 5969.0, (1, 2): 5358.0, (1, 4): 5091.0}  # read:write
P_MFMA = 54.0e12     # FP64 matrix-core flops/s (best kernel's executed rate; probe 51.5)
# fraction of P_MFMA reached with this many waves per SIMD (peak probe: one
# wave keeps the FP64 matrix core busy 48% of the cycles, two or more 66%)
MFMA_BY_WAVES = {1: 0.48 / 0.66, 2: 1.0}
P_VALU = 66.0e12     # FP64 vector FMA flops/s at full occupancy (probe)
T_LAUNCH = 6e-6      # a launch plus, for TSMTTSM, the fold of the partials
CUS = 256
WAVE_SLOTS = 8       # waves per SIMD


def bandwidth(q):
    """Read bandwidth (B/s) with q bytes in flight per CU (Table-1 interpolation)."""
    xs = [x for x, _ in TABLE1]
    if q <= xs[0]:
        return TABLE1[0][1] * 1e9 * q / xs[0]
    i = bisect.bisect_left(xs, q)
    if i >= len(xs):
        return TABLE1[-1][1] * 1e9
    (x0, y0), (x1, y1) = TABLE1[i - 1], TABLE1[i]
    return (y0 + (y1 - y0) * (math.log(q) - math.log(x0)) / (math.log(x1) - math.log(x0))) * 1e9


def mix_ceiling(M, N):
    """Bandwidth ceiling (B/s) of TSMM's stream: A read (M columns), B written (N columns)."""
    r = M / float(N)
    best = min(MIX_CEILING, key=lambda k: abs(math.log(k[0] / k[1]) - math.log(r)))
    return MIX_CEILING[best] * 1e9


def _cw(dt):
    return 2 if dt in ("c128", "c64", "c64a") else 1


def _elem(dt):
    return {"r64": 8, "c128": 16, "r32": 4, "c64": 8, "r32a": 4, "c64a": 8}[dt]


def rows_ahead(v):
    """Rows of A (and B) one block has requested ahead of its multiplications."""
    c = v["cfg"]
    nbuf = c.get("NBUF", 2)
    if c["kind"] == "lds":
        return c["RT"]
    if c["kind"] == "dot":
        return 128 * c["U"] * c["WPB"] * (nbuf - 1)
    if c["kind"] == "packed":
        per = (4 if v["op"] == "tsmttsm" else 16) * c["U"] * c["WPB"]
        P = max(1, 16 // max(v["M"], v["N"])) if v["op"] == "tsmttsm" else max(1, 16 // v["N"])
        return per * P * (nbuf - 1)
    if c["kind"] == "valu":
        return 64 * c["U"] * c["WPB"] * (nbuf - 1)
    if v["op"] == "tsmttsm":
        return 4 * c["U"] * (c["WPB"] // c.get("MW", 1)) * (nbuf - 1)
    return 16 * c["U"] * c["WPB"] * (nbuf - 1)


def blocks_per_cu(v, res):
    """Resident blocks per CU: the compiler's register-limited waves per SIMD
    (resource records) and the LDS the block uses."""
    c = v["cfg"]
    wpb = c["WPB"]
    occ = (res or {}).get("occupancy", WAVE_SLOTS)
    by_regs = max(1, occ * 4 // wpb)
    lds = (res or {}).get("lds")
    if lds is None and c["kind"] == "lds":
        cw = _cw(v["dt"])
        lds = max(2 * c["RT"] * (v["M"] + v["N"]) * cw * 8, v["M"] * v["N"] * cw * 8)
    by_lds = (160 << 10) // lds if lds else by_regs
    return max(1, min(by_regs, by_lds, WAVE_SLOTS * 4 // wpb))


def waves_per_simd(v, res):
    """Resident waves per SIMD of the kernel."""
    return max(1, blocks_per_cu(v, res) * v["cfg"]["WPB"] // 4)


def executed_flops(v, K):
    """FP64 flops the kernel executes: matrix-core kinds on padded 16 x 16 x 4
    fragments, complex three-product form 6MNK."""
    c = v["cfg"]
    M, N = v["M"], v["N"]
    cplx = _cw(v["dt"]) == 2
    mult = (6 if c.get("G3") else 8) if cplx else 2
    if c["kind"] in ("mfma", "lds", "a32") and v["op"] == "tsmttsm":
        Mp, Np = 16 * -(-M // 16), 16 * -(-N // 16)
        return mult * Mp * Np * K, 0.0
    if c["kind"] in ("mfma", "a32"):
        Mp, Np = 4 * -(-M // 4), 16 * -(-N // 16)
        return mult * Mp * Np * K, 0.0
    if c["kind"] == "packed":
        P = max(1, 16 // max(M, N)) if v["op"] == "tsmttsm" else max(1, 16 // N)
        return mult * 16 * 16 * K / P, 0.0
    return 0.0, mult * M * N * K


def predict(v, K, res=None):
    """Predicted seconds of one call of variant v at K rows."""
    M, N = v["M"], v["N"]
    s = _elem(v["dt"])
    byts = s * K * (M + N) + 8 * _cw(v["dt"]) * M * N
    q = blocks_per_cu(v, res) * rows_ahead(v) * s * (M + (N if v["op"] == "tsmttsm" else 0))
    bw = bandwidth(q)
    if v["op"] == "tsmm":
        bw = min(bw, mix_ceiling(M, N))
    fm, fv = executed_flops(v, K)
    # binary32 products (the a32 kernels and the LDS-staged kernel of the
    # binary32-arithmetic types) run at twice the binary64 matrix-core rate
    p_mfma = P_MFMA * (2.0 if v["dt"] in ("r32a", "c64a") and v["cfg"]["kind"] in ("a32", "lds") else 1.0)
    p_mfma *= MFMA_BY_WAVES.get(waves_per_simd(v, res), 1.0)
    return max(byts / bw, fm / p_mfma, fv / P_VALU) + T_LAUNCH


def prune(variants, K, resources=None, keep=1.3):
    """The variants whose prediction is within `keep` x the best prediction."""
    pred = {id(v): predict(v, K, (resources or {}).get(_name(v))) for v in variants}
    best = min(pred.values())
    return [v for v in variants if pred[id(v)] <= keep * best]


def _name(v):
    from paper_1905_03136_amd import codegen
    return codegen.variant_name(v)


def _spearman(xs, ys):
    def ranks(a):
        order = sorted(range(len(a)), key=lambda i: a[i])
        r = [0.0] * len(a)
        for k, i in enumerate(order):
            r[i] = k
        return r
    rx, ry = ranks(xs), ranks(ys)
    n = len(xs)
    if n < 3:
        return float("nan")
    mx, my = sum(rx) / n, sum(ry) / n
    num = sum((a - mx) * (b - my) for a, b in zip(rx, ry))
    den = math.sqrt(sum((a - mx) ** 2 for a in rx) * sum((b - my) ** 2 for b in ry))
    return num / den if den else float("nan")


def evaluate(db_paths, resources=None, keep=1.3):
    """Per (op, dtype, M, N) of the databases: rank correlation of predicted and
    measured times, whether the measured fastest survives pruning at `keep`,
    the fraction of candidates pruned, and the slowdown of the fastest survivor
    against the measured fastest."""
    recs = {}
    for p in db_paths:
        with open(p) as f:
            for line in f:
                try:
                    r = json.loads(line)
                except ValueError:
                    continue
                if r.get("ok") and r.get("us") and r.get("M"):
                    recs[(r["op"], r["dt"], r["M"], r["N"], r["name"])] = r
    groups = collections.defaultdict(list)
    for (op, dt, M, N, _), r in recs.items():
        groups[(op, dt, M, N)].append(r)
    rows = []
    for key, rs in sorted(groups.items()):
        if len(rs) < 3:
            continue
        op, dt, M, N = key
        vs = [dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=r["cfg"]) for r in rs]
        pred = [predict(v, r["K"], (resources or {}).get(r["name"])) for v, r in zip(vs, rs)]
        meas = [r["us"] for r in rs]
        best_p = min(pred)
        kept = [i for i in range(len(rs)) if pred[i] <= keep * best_p]
        best_m = min(meas)
        rows.append(dict(op=op, dt=dt, M=M, N=N, candidates=len(rs), kept=len(kept),
                         rho=_spearman(pred, meas), best_kept=any(meas[i] == best_m for i in kept),
                         slowdown=min(meas[i] for i in kept) / best_m))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    e = sub.add_parser("evaluate")
    e.add_argument("--db", action="append", required=True)
    e.add_argument("--keep", type=float, default=1.3)
    e.add_argument("--tag", default="tune", help="build whose resource records give register use")
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1905_03136_amd import build, codegen
    rows = []
    for p in a.db:
        with open(p) as f:
            for line in f:
                try:
                    r = json.loads(line)
                except ValueError:
                    continue
                if r.get("M"):
                    rows.append(dict(op=r["op"], dt=r["dt"], M=r["M"], N=r["N"], maxM=r["M"], maxN=r["N"], cfg=r["cfg"]))
    res = build.variant_resources(rows, tag="_" + a.tag)
    out = evaluate(a.db, res, a.keep)
    print("| op | dtype | M x N | candidates | kept | rank corr. | fastest kept | fastest kept / fastest |")
    print("|---|---|---|---:|---:|---:|---|---:|")
    for r in out:
        print("| %s | %s | %dx%d | %d | %d | %.2f | %s | %.3f |" % (r["op"], r["dt"], r["M"], r["N"], r["candidates"],
                                                                 r["kept"], r["rho"], "yes" if r["best_kept"] else "no",
                                                                 r["slowdown"]))
    n = len(out)
    if n:
        print()
        print("%d widths: fastest kept in %d, median kept fraction %.2f, geometric-mean slowdown of the pruned "
              "search %.3f, median rank correlation %.2f" % (
                  n, sum(r["best_kept"] for r in out),
                  sorted(r["kept"] / r["candidates"] for r in out)[n // 2],
                  math.exp(sum(math.log(r["slowdown"]) for r in out) / n),
                  sorted(r["rho"] for r in out if r["rho"] == r["rho"])[n // 2]))


if __name__ == "__main__":
    main()
