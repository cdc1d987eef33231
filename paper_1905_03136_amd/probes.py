"""Machine probes: the paper's Table 1 grid (bandwidth against occupancy and
loads in flight), read:write mixes of the two products, the peak arithmetic
rates, and memory latency by pointer chasing (Section 1.6, Table 1; Section
5.3 applies Little's law to the measured latency).  Every probe is a kernel
of the library (tsg_stream_probe, tsg_peak_probe, tsg_latency_probe); this
module only allocates buffers, times the launches with events and prints.

    python -m paper_1905_03136_amd.probes [--out probes.json]
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

GiB = 1 << 30


def _time(fn, reps=5, warmup=1):
    """Median seconds of fn() over reps launches (events on the current stream)."""
    import torch
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e-3)
    ts.sort()
    return ts[len(ts) // 2]


def table1(x, occs=(1, 2, 4, 8, 16), ilps=(1, 2, 4, 8, 16)):
    """Read-only bandwidth (GB/s) over blocks of 256 threads per CU x loads in flight."""
    import torch
    from paper_1905_03136_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    out = {}
    for occ in occs:
        for ilp in ilps:
            moved = [0]

            def run():
                st, moved[0] = _lib.tsg_stream_probe(x.data_ptr(), x.numel(), None, 0, occ, ilp, 1, s)
                _lib.check(st)
            t = _time(run)
            out["%d,%d" % (occ, ilp)] = moved[0] / t / 1e9
            print("[probe] read  blocks/CU %2d  loads in flight %2d: %7.0f GB/s" % (occ, ilp, out["%d,%d" % (occ, ilp)]),
                  flush=True)
    return out


def mixes(x, y, ratios=((1, 0), (1, 1), (4, 1), (1, 4), (2, 1), (1, 2)), occs=(2, 4, 8), ilps=(4, 8, 16)):
    """Best read+write bandwidth (GB/s) per write:read ratio, with streaming
    and with cached stores; the configurations tried and the best one."""
    import torch
    from paper_1905_03136_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    out = {}
    for rd, wr in ratios:
        xb = x.numel() if rd >= wr else x.numel() * rd // wr
        yb = xb * wr // rd
        for nt in ((1, 0) if wr else (1,)):
            best = (0.0, None)
            for occ in occs:
                for ilp in ilps:
                    moved = [0]

                    def run():
                        st, moved[0] = _lib.tsg_stream_probe(x.data_ptr(), xb, y.data_ptr() if wr else None, yb,
                                                             occ, ilp, nt, s)
                        _lib.check(st)
                    t = _time(run)          # runs the probe, which sets moved[0]
                    bw = moved[0] / t / 1e9
                    if bw > best[0]:
                        best = (bw, (occ, ilp))
            key = "%d:%d %s" % (rd, wr, "streaming" if nt else "cached")
            out[key] = {"GBps": best[0], "blocks_per_cu": best[1][0], "loads_in_flight": best[1][1]}
            print("[probe] read:write %d:%d %-9s stores: %7.0f GB/s (blocks/CU %d, loads in flight %d)"
                  % (rd, wr, "streaming" if nt else "cached", best[0], best[1][0], best[1][1]), flush=True)
    return out


def peaks(occs=(1, 2, 4, 8), iters=20000):
    """Arithmetic rates (TF/s) of the peak kernels per blocks of 256 threads per CU."""
    import torch
    from paper_1905_03136_amd import _lib
    s = torch.cuda.current_stream().cuda_stream
    names = {_lib.TSG_PEAK_MFMA_F64: "mfma_f64", _lib.TSG_PEAK_VALU_F64: "valu_f64",
             _lib.TSG_PEAK_MFMA_F32: "mfma_f32", _lib.TSG_PEAK_MIXED_F64: "mixed_f64"}
    out = {}
    for kind, name in names.items():
        out[name] = {}
        for occ in occs:
            fl = [0.0]

            def run():
                st, fl[0] = _lib.tsg_peak_probe(kind, occ, iters, s)
                _lib.check(st)
            t = _time(run, reps=3)      # runs the probe, which sets fl[0]
            rate = fl[0] / t / 1e12
            out[name][str(occ)] = rate
            print("[probe] %-9s blocks/CU %d: %6.1f TF/s" % (name, occ, rate), flush=True)
    return out


def latency(sizes=(1 << 20, 64 << 20, 4 * GiB), steps=20000, stride_bytes=256):
    """Cycles and ns per dependent load of a random cycle over each working set
    (one element per stride_bytes, so each load touches its own line)."""
    import numpy as np
    import torch
    from paper_1905_03136_amd import _lib
    dev = torch.device("cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    out = {}
    for ws in sizes:
        step = stride_bytes // 8
        n = ws // stride_bytes
        perm = np.random.default_rng(5).permutation(n)
        nxt = np.zeros(n * step, dtype=np.int64)
        # the cycle visits element perm[0] -> perm[1] -> ... -> perm[n-1] -> perm[0], spaced by the stride
        nxt[perm * step] = np.roll(perm, -1) * step
        d = torch.from_numpy(nxt).to(dev)
        res = torch.zeros(3, dtype=torch.int64, device=dev)
        _lib.check(_lib.tsg_latency_probe(d.data_ptr(), steps, res.data_ptr(), s))
        torch.cuda.synchronize()
        cyc, ticks, _ = res.cpu().tolist()
        ns = ticks * 10.0 / steps           # 100 MHz constant clock
        out[str(ws)] = {"cycles": cyc / steps, "ns": ns}
        print("[probe] latency at %8.1f MiB: %6.0f cycles, %6.0f ns per load" % (ws / 2 ** 20, cyc / steps, ns),
              flush=True)
        del d
    return out


def markdown(res):
    """Tables of a probe run's JSON (no GPU needed)."""
    out = []
    t1 = res["table1"]
    occs = sorted({int(k.split(",")[0]) for k in t1})
    ilps = sorted({int(k.split(",")[1]) for k in t1})
    out.append("**Read bandwidth (GB/s) against blocks of 256 threads per CU (rows) and 16-byte loads in flight "
               "per thread (columns)** -- the paper's Table 1 grid\n")
    out.append("| blocks/CU \\\\ loads | " + " | ".join(str(i) for i in ilps) + " |")
    out.append("|---|" + "---:|" * len(ilps))
    for o in occs:
        out.append("| %d | " % o + " | ".join("%.0f" % t1["%d,%d" % (o, i)] for i in ilps) + " |")
    out.append("\n**Read:write mixes** (bytes read : bytes written; best launch shape of the probe)\n")
    out.append("| mix | GB/s (read + write) | blocks/CU | loads in flight |")
    out.append("|---|---:|---:|---:|")
    for k, v in res["mixes"].items():
        out.append("| %s | %.0f | %d | %d |" % (k, v["GBps"], v["blocks_per_cu"], v["loads_in_flight"]))
    out.append("\n**Peak arithmetic (TFLOP/s) against blocks of 256 threads per CU**\n")
    pk = res["peaks"]
    cols = sorted({int(b) for v in pk.values() for b in v})
    out.append("| unit | " + " | ".join(str(c) for c in cols) + " |")
    out.append("|---|" + "---:|" * len(cols))
    for k, v in pk.items():
        out.append("| %s | " % k + " | ".join("%.1f" % v[str(c)] if str(c) in v else "" for c in cols) + " |")
    out.append("\n**Load latency by pointer chasing** (one lane, dependent loads over a working set)\n")
    out.append("| working set | cycles | ns |")
    out.append("|---:|---:|---:|")
    for k, v in sorted(res["latency"].items(), key=lambda kv: int(kv[0])):
        out.append("| %.0f MiB | %.0f | %.0f |" % (int(k) / 2 ** 20, v["cycles"], v["ns"]))
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="probes.json")
    ap.add_argument("--gib", type=int, default=4, help="GiB streamed by the bandwidth probes")
    ap.add_argument("--markdown", default="", help="no GPU: print the tables of a probe run's JSON file and exit")
    a = ap.parse_args(argv)
    if a.markdown:
        with open(a.markdown) as f:
            print(markdown(json.load(f)), end="")
        return
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x = torch.empty(a.gib * GiB, dtype=torch.uint8, device=dev)
    x.view(torch.float64).uniform_(-1, 1)
    y = torch.empty(a.gib * GiB, dtype=torch.uint8, device=dev)
    res = {"table1": table1(x), "mixes": mixes(x, y), "peaks": peaks(), "latency": latency()}
    del x, y
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    print("[probe] wrote %s" % a.out, flush=True)


if __name__ == "__main__":
    main()
