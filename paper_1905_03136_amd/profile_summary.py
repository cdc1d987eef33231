"""Summarise rocprofv3 output of a bench run into a short markdown file.

Inputs are the directories rocprofv3 wrote for three runs of the same bench
command: a kernel trace (``--kernel-trace --stats``) and two counter passes
(``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``).  The counters are reported
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


def counters(d, counter):
    """Per kernel (full name): list of counter values in bytes (the counter
    is in KiB), in dispatch order."""
    out = collections.defaultdict(list)
    cur = _db(d).cursor()
    for name, value in cur.execute("select kernel_name, value from counters_collection where counter_name = ? "
                                   "order by dispatch_id", (counter,)):
        out[name].append(float(value) * 1024.0)
    return out


def _probe(vals, key):
    hits = [v for k, v in vals.items() if key in k]
    if not hits:
        raise ValueError("no %s dispatch in the counter run" % key)
    xs = sorted(hits[0])
    return xs[len(xs) // 2]


def summarise(trace, fetch, write, bench_json, command, probe_bytes):
    stats = kernel_stats(trace)
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
        rows.append(dict(s, read=rd, written=wr))
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
    ap.add_argument("--bench-json", default="")
    ap.add_argument("--command", action="append", default=[], help="a command line that produced the data")
    ap.add_argument("--probe-bytes", type=float, default=float(8 << 30))
    ap.add_argument("--title", default="Kernel profile")
    ap.add_argument("--out", required=True)
    ap.add_argument("--no-dominant", action="store_true",
                    help="omit the dominant kernel's per-launch record (runs that launch a kernel at several sizes)")
    a = ap.parse_args(argv)
    rows, fs, ws, bench, roof = summarise(a.trace, a.fetch, a.write, a.bench_json, a.command, a.probe_bytes)
    with open(a.out, "w") as f:
        f.write(render(rows, fs, ws, bench, roof, a.command, a.title, dominant=not a.no_dominant))
    print("wrote %s" % a.out)


if __name__ == "__main__":
    main()
