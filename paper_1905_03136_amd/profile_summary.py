"""Summarise rocprofv3 output of a bench run into a short markdown file.

Inputs are the directories rocprofv3 wrote for runs of the same bench
command: a kernel trace (``--kernel-trace --stats``), two counter passes
(``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``) and optionally a pass with
the FP64 instruction counters (``ARITH``), from which the executed FP64
matrix-core and vector rates of every kernel follow.  The counters are reported
in KiB per dispatch and do not count every byte as the algorithm does, so
each is scaled by what it reads for the library's own stream probes of known
size (``tsg::stream_read`` reads, ``tsg::stream_copy`` reads and writes, a
fixed number of bytes per launch): scale = known bytes / counted bytes.

The markdown ends with a JSON block (kernel, average duration, scaled HBM
bytes per launch, the source hash of the kernels profiled) that bench.py
uses as the roofline record's ``traffic`` while the kernel sources still
have that hash.

    python -m paper_1905_03136_amd.profile_summary --trace DIR --fetch DIR --write DIR \\
        --bench-json FILE --command "..." --out profiles/NAME.md
"""
import argparse
import collections
import sqlite3
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash():
    """Hash of everything that decides which code the TSMTTSM / TSMM calls
    run: their kernel templates and device helpers, the runtime (variant
    choice, grid sizing), the code generator and the tuned table.  The batched
    form and the bandwidth probes have sources of their own and are not part
    of it."""
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.hpp"))
                   if os.path.basename(f) not in ("tsg_batched.hip", "tsg_stream.hip"))
    files += [os.path.join(HERE, "codegen.py"), os.path.join(HERE, "tuned.json")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    if "at::native" in name or "distribution" in name:
        return "torch (input generation / copies)"
    n = name.replace("void ", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0]


def _one(d, suffix):
    got = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not got:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return got[0]


def _db(d):
    """rocprofv3's default output: one SQLite database (rocpd schema) per run."""
    return sqlite3.connect(_one(d, "_results.db"))


def kernel_stats(d):
    """Per kernel: dispatch count, average duration and share of the total kernel time."""
    cur = _db(d).cursor()
    rows = cur.execute("select name, count(*), avg(duration), sum(duration) from kernels group by name").fetchall()
    total = sum(r[3] for r in rows) or 1
    out = [dict(name=short(n), full=n, calls=int(c), avg_us=float(a) / 1e3, pct=100.0 * s / total)
           for n, c, a, s in rows]
    return sorted(out, key=lambda r: -r["pct"])


def counters(d, counter, scale=1024.0):
    """Per kernel (full name): list of counter values in dispatch order,
    times `scale` (1024: the size counters are in KiB)."""
    out = collections.defaultdict(list)
    cur = _db(d).cursor()
    for name, value in cur.execute("select kernel_name, value from counters_collection where counter_name = ? "
                                   "order by dispatch_id", (counter,)):
        out[name].append(float(value) * scale)
    return out


# FP64 instruction counters of the arithmetic pass (wave-level instruction counts)
ARITH = ["SQ_INSTS_VALU_MFMA_F64", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
         "SQ_INSTS_VALU_MUL_F64", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU",
         "GRBM_GUI_ACTIVE"]


def arith(dirs, avg_us):
    """Per kernel: average counter values per dispatch and the executed FP64
    rates they give with the kernel's average duration `avg_us` (from the
    trace): every FP64 matrix-core instruction the library issues is a
    16x16x4 product (2048 flops per wave instruction), every FP64 FMA
    128 flops per wave instruction (64 lanes), an add or multiply 64."""
    vals = {c: {} for c in ARITH}
    for d in dirs:
        for c in ARITH:
            got = counters(d, c, 1.0)
            if got:
                vals[c] = got
    out = {}
    names = set()
    for v in vals.values():
        names |= set(v)
    for n in names:
        avg = {c: (sum(vals[c][n]) / len(vals[c][n]) if vals[c].get(n) else None) for c in ARITH}
        t = avg_us.get(n)
        rec = dict(avg)
        if t:
            mf = (avg["SQ_INSTS_VALU_MFMA_F64"] or 0) * 2048.0
            vf = (avg["SQ_INSTS_VALU_FMA_F64"] or 0) * 128.0 + ((avg["SQ_INSTS_VALU_ADD_F64"] or 0) +
                                                                  (avg["SQ_INSTS_VALU_MUL_F64"] or 0)) * 64.0
            rec.update(mfma_tflops=mf / (t * 1e-6) / 1e12, valu_tflops=vf / (t * 1e-6) / 1e12)
        out[n] = rec
    return out


def _probe(vals, key):
    hits = [v for k, v in vals.items() if key in k]
    if not hits:
        raise ValueError("no %s dispatch in the counter run" % key)
    xs = sorted(hits[0])
    return xs[len(xs) // 2]


def summarise(trace, fetch, write, bench_json, command, probe_bytes, arith_dir=None):
    stats = kernel_stats(trace)
    ar = arith(arith_dir, {s["full"]: s["avg_us"] for s in stats}) if arith_dir else {}
    fv = counters(fetch, "FETCH_SIZE")
    wv = counters(write, "WRITE_SIZE")
    f_scale = probe_bytes / _probe(fv, "stream_read")
    w_scale = probe_bytes / _probe(wv, "stream_copy")
    bench = json.load(open(bench_json)) if bench_json else {}
    roof = bench.get("roofline", {})
    rows = []
    for s in stats:
        f = fv.get(s["full"], [])
        w = wv.get(s["full"], [])
        rd = sum(f) / len(f) * f_scale if f else None
        wr = sum(w) / len(w) * w_scale if w else None
        rows.append(dict(s, read=rd, written=wr, arith=ar.get(s["full"])))
    return rows, f_scale, w_scale, bench, roof


def render(rows, f_scale, w_scale, bench, roof, commands, title, dominant=True):
    lines = ["# %s" % title, "", "Commands (run from the repository root on one MI355X):", ""]
    lines += ["    " + c for c in commands]
    lines += ["", "Counter scale factors from the stream probes of known size: FETCH_SIZE x %.3f, "
              "WRITE_SIZE x %.3f (bytes per counted byte)." % (f_scale, w_scale), "",
              "| kernel | calls | avg us | % time | HBM read MB/launch | HBM write MB/launch |",
              "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        if r["pct"] < 0.05 and "tsg" not in r["full"] and "orth" not in r["full"]:
            continue
        lines.append("| `%s` | %d | %.1f | %.2f | %s | %s |" % (
            r["name"][:110], r["calls"], r["avg_us"], r["pct"],
            "%.1f" % (r["read"] / 1e6) if r["read"] is not None else "-",
            "%.1f" % (r["written"] / 1e6) if r["written"] is not None else "-"))
    if any(r.get("arith") for r in rows):
        lines += ["", "FP64 arithmetic per kernel (counter pass: wave-level instruction counts per dispatch; "
                  "executed rate = instructions x flops per instruction / trace duration; matrix core: 2048 "
                  "flops per 16x16x4 FP64 product, vector: 128 per FMA, 64 per add or multiply):", "",
                  "| kernel | MFMA F64 insts | MFMA MOPS F64 | VALU FMA F64 | VALU add+mul F64 | executed MFMA TF/s "
                  "| executed VALU TF/s | MFMA busy cycles | SQ busy cycles | GRBM GUI active |",
                  "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
        for r in rows:
            a = r.get("arith")
            if not a or not (a.get("SQ_INSTS_VALU_MFMA_F64") or a.get("SQ_INSTS_VALU_FMA_F64")):
                continue
            f = lambda x: "-" if x is None else "%.4g" % x
            lines.append("| `%s` | %s | %s | %s | %s | %s | %s | %s | %s | %s |" % (
                r["name"][:90], f(a["SQ_INSTS_VALU_MFMA_F64"]), f(a["SQ_INSTS_VALU_MFMA_MOPS_F64"]),
                f(a["SQ_INSTS_VALU_FMA_F64"]), f((a["SQ_INSTS_VALU_ADD_F64"] or 0) + (a["SQ_INSTS_VALU_MUL_F64"] or 0)),
                "%.1f" % a.get("mfma_tflops", 0), "%.1f" % a.get("valu_tflops", 0),
                f(a["SQ_VALU_MFMA_BUSY_CYCLES"]), f(a["SQ_BUSY_CYCLES"]), f(a["GRBM_GUI_ACTIVE"])))
    rec = None
    kern = roof.get("kernel_symbol") if dominant else None
    if not dominant:
        lines += ["", "No per-launch record of the bench's dominant kernel here: this run launches some kernels "
                  "at more than one size, and the per-launch figures above average over them."]
    if kern:
        hit = [r for r in rows if r["full"].startswith(kern + "(")]
        if hit and hit[0]["read"] is not None and hit[0]["written"] is not None:
            h = hit[0]
            rec = {"kernel": kern, "kernel_variant": roof.get("kernel"), "avg_us": round(h["avg_us"], 2), "read_bytes": round(h["read"]),
                   "write_bytes": round(h["written"]), "traffic": round(h["read"] + h["written"]),
                   "bench_avg_us": roof.get("avg_us"), "algorithmic_bytes": roof.get("bytes"),
                   "source_hash": bench.get("source_hash")}
            if h.get("arith") and "mfma_tflops" in h["arith"]:
                rec.update(executed_mfma_tflops=round(h["arith"]["mfma_tflops"], 2),
                           executed_valu_tflops=round(h["arith"]["valu_tflops"], 2),
                           mfma_f64_insts=h["arith"]["SQ_INSTS_VALU_MFMA_F64"],
                           valu_fma_f64_insts=h["arith"]["SQ_INSTS_VALU_FMA_F64"])
    if rec:
        lines += ["", "Dominant kernel of the bench step: `%s`: %.1f us per launch in the trace (bench's own "
                  "events: %s us); HBM traffic %.1f MB per launch against %.1f MB algorithmic." % (
                      short(rec["kernel"]), rec["avg_us"], rec["bench_avg_us"], rec["traffic"] / 1e6,
                      (rec["algorithmic_bytes"] or 0) / 1e6)]
    lines += ["", "```json", json.dumps({"dominant": rec}, indent=1), "```", ""]
    return "\n".join(lines)


def traffic_record(path, kernel, src_hash):
    """The JSON block of a summary, if it is for ``kernel`` and sources with
    hash ``src_hash``; else None."""
    try:
        text = open(path).read()
    except OSError:
        return None
    if "```json" not in text:
        return None
    block = text.split("```json", 1)[1].split("```", 1)[0]
    try:
        rec = json.loads(block).get("dominant")
    except ValueError:
        return None
    if not rec or rec.get("kernel") != kernel or rec.get("source_hash") != src_hash:
        return None
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--arith", action="append", default=[],
                    help="directory of a counter pass with some of the FP64 instruction counters (repeatable)")
    ap.add_argument("--bench-json", default="")
    ap.add_argument("--command", action="append", default=[], help="a command line that produced the data")
    ap.add_argument("--probe-bytes", type=float, default=float(8 << 30))
    ap.add_argument("--title", default="Kernel profile")
    ap.add_argument("--out", required=True)
    ap.add_argument("--no-dominant", action="store_true",
                    help="omit the dominant kernel's per-launch record (runs that launch a kernel at several sizes)")
    a = ap.parse_args(argv)
    rows, fs, ws, bench, roof = summarise(a.trace, a.fetch, a.write, a.bench_json, a.command, a.probe_bytes,
                                          a.arith or None)
    with open(a.out, "w") as f:
        f.write(render(rows, fs, ws, bench, roof, a.command, a.title, dominant=not a.no_dominant))
    print("wrote %s" % a.out)


if __name__ == "__main__":
    main()
