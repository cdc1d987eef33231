"""Autotuner: exhaustive timing of the generated configurations.

The paper picks the best configuration of every matrix size by an exhaustive
search over the generator's options (Section 5.1; Sections 6.1-6.3 show the
cross sections of that search).  Here the candidate space of a width comes
from ``codegen.candidates`` (mapping, rows in flight, waves per block, wave
split of C), already pruned by a register model.

    python -m paper_1905_03136_amd.tune build            # CPU: compile every candidate
    python -m paper_1905_03136_amd.tune run --db DB.jsonl --out tuned.json   # GPU

``run`` times each candidate at K rows (default 2^24), rotating through
enough disjoint buffer sets that consecutive calls never find their data in
the 256 MB Infinity Cache.  Before it is timed, every candidate must equal the
exact product of integer-valued inputs, computed on the host in int64
arithmetic (the inputs' products and sums are exact in binary64, and in the
binary32-arithmetic kernels' 32-row stretches), bit for bit, both on the full
grid and on a grid of three blocks (every block then works through many
tiles); a candidate that differs is recorded as failed and never chosen.  Records are appended to a JSONL
database, so an interrupted run resumes where it stopped; ``tuned.json``
keeps the fastest correct configuration per (operation, dtype, M, N) and is
read by the code generator when the product library is built.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TUNE_LIB = os.path.join(HERE, "libtsgemm_tune.so")
HBM_PEAK = 8.0e12
FP64_PEAK = 78.6e12


def _widths(name):
    from paper_1905_03136_amd import codegen
    if name == "graded":
        return codegen.GRADED
    if name == "square":
        return codegen.SQUARE_ALL
    if name == "narrow":
        return codegen.NARROW
    out = []
    for tok in name.split(","):
        m, n = tok.split("x")
        out.append((int(m), int(n)))
    return out


def cmd_build(args):
    """Compile the candidates of the selected widths, operations and dtypes
    into a tuning library.  --kinds keeps only candidates of those mappings
    (plus, with --with-tuned, each width's configuration in the current
    table, so that a partial search re-times the incumbent beside them);
    --tag builds a library of its own (_build/libtsgemm_<tag>.so, for
    TSG_LIBRARY) without touching the default tuning library."""
    sys.path.insert(0, ROOT)
    from paper_1905_03136_amd import build, codegen
    lib = TUNE_LIB if not args.tag else build.tagged_lib(args.tag)
    if args.generic:
        # the run-time-width classes' candidates (plus the product's own
        # run-time-width variants, so that every pair has a kernel)
        variants, names = [], set()
        for v in generic_tuning_variants() + codegen.generic_variants():
            if codegen.variant_name(v) not in names:
                names.add(codegen.variant_name(v))
                variants.append(v)
        build.build(variants=variants, lib_path=lib, tag="_" + (args.tag or "tune"))
        return
    variants = codegen.tuning_variants(_widths(args.widths))
    ops = set(args.ops.split(",")) if args.ops else None
    dtypes = set(args.dtypes.split(",")) if args.dtypes else None
    kinds = set(args.kinds.split(",")) if args.kinds else None
    tuned = codegen.load_tuned(os.path.join(HERE, "tuned.json")) if args.with_tuned else {}

    def keep(v):
        if v["M"] == 0:
            return True  # run-time-width variants always
        if (ops and v["op"] not in ops) or (dtypes and v["dt"] not in dtypes):
            return False
        if kinds is None or v["cfg"]["kind"] in kinds:
            return True
        return tuned.get((v["op"], v["dt"], v["M"], v["N"])) == v["cfg"]
    variants = [v for v in variants if keep(v)]
    names = {codegen.variant_name(v) for v in variants}
    # the incumbent of a width need not be among the enumerated candidates
    for key, cfg in tuned.items():
        if len(key) != 4:
            continue
        op, dt, M, N = key
        if (ops and op not in ops) or (dtypes and dt not in dtypes) or (M, N) not in _widths(args.widths):
            continue
        v = dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=cfg)
        if codegen.variant_name(v) not in names:
            names.add(codegen.variant_name(v))
            variants.append(v)
    build.build(variants=variants, lib_path=lib, tag="_" + (args.tag or "tune"))


def exact_product(op, A, B):
    """op(A)^T B ("tsmttsm") or A B ("tsmm") of integer-valued numpy arrays in
    int64 arithmetic (complex: the real expansion), returned as float64 or
    complex128.  Independent of the oracle and of the library."""
    import numpy as np
    mul = (lambda x, y: x.T @ y) if op == "tsmttsm" else (lambda x, y: x @ y)
    if not np.iscomplexobj(A):
        return mul(A.astype(np.int64), B.astype(np.int64)).astype(np.float64)
    ar, ai = A.real.astype(np.int64), A.imag.astype(np.int64)
    br, bi = B.real.astype(np.int64), B.imag.astype(np.int64)
    re = mul(ar, br) - mul(ai, bi)
    im = mul(ar, bi) + mul(ai, br)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def _algorithmic(op, cplx, K, M, N, real_bytes=8):
    """Eq. 1 bytes (tall matrices in the storage type, C in binary64) and flops."""
    s = (2 if cplx else 1) * real_bytes
    c = 16 if cplx else 8
    return s * (K * M + K * N) + c * M * N, (8 if cplx else 2) * M * N * K


class _Timer:
    """Forced variants timed on one (op, dtype, M, N) at K rows: each must
    give the exact product of an integer-valued problem (on the full grid and
    on three blocks), then the median of ``reps`` calls, rotating over buffer
    sets of at least 1 GiB in all so that no call finds its operands in the
    caches."""

    def __init__(self, K, warmup, reps):
        import torch
        from paper_1905_03136_amd import _lib
        self.torch, self.K, self.warmup, self.reps = torch, K, warmup, reps
        self.dev = torch.device("cuda:0")
        torch.cuda.set_device(self.dev)
        self.names = {_lib.tsg_variant_name(i) for i in range(_lib.tsg_variant_count())}
        self.pools = {}
        for cplx in (False, True):
            t = torch.empty(2 * K * 64 * (2 if cplx else 1), dtype=torch.float64, device=self.dev)
            g = torch.Generator(device=self.dev)
            g.manual_seed(1234 + int(cplx))
            t.uniform_(-1.0, 1.0, generator=g)
            self.pools[cplx] = t

    def measure(self, op, dt, M, N, variants, base=None):
        """One record per variant (``base`` merged into each)."""
        torch = self.torch
        from paper_1905_03136_amd import _lib, api, codegen, inputs
        K, dev = self.K, self.dev
        cplx = codegen.DTYPES[dt][1]
        f32 = codegen.is_f32(dt)
        cw = 2 if cplx else 1
        tdt = torch.complex128 if cplx else torch.float64            # small matrix C
        sdt = (torch.complex64 if cplx else torch.float32) if f32 else tdt  # storage of A, B
        # integer-valued problem: every candidate must give the exact product
        kc = 4099
        Ah = inputs.host_integers(kc, M, 7, inputs.STREAM_A, cplx)
        Bh = inputs.host_integers(kc, N, 7, inputs.STREAM_B, cplx)
        Xh = inputs.host_integers(M, N, 7, inputs.STREAM_C, cplx)
        exact = torch.from_numpy(exact_product(op, Ah, Bh if op == "tsmttsm" else Xh)).to(dev)
        Ai = torch.from_numpy(Ah).to(dev).to(sdt)
        Bi = torch.from_numpy(Bh).to(dev).to(sdt)
        Xi = torch.from_numpy(Xh).to(dev)
        # buffer sets for timing (pool reinterpreted as binary32 for the precision form)
        pool = self.pools[cplx].view(torch.float32) if f32 else self.pools[cplx]
        ws_elems = K * (M + N) * cw
        ws_bytes = ws_elems * pool.element_size()
        R = max(1, min(int(math.ceil((1 << 30) / ws_bytes)), pool.numel() // ws_elems))
        sets = []
        for r in range(R):
            chunk = pool[r * ws_elems:(r + 1) * ws_elems]
            a = chunk[:K * M * cw]
            b = chunk[K * M * cw:]
            if cplx:
                a = torch.view_as_complex(a.view(K, M, 2))
                b = torch.view_as_complex(b.view(K, N, 2))
            else:
                a = a.view(K, M)
                b = b.view(K, N)
            sets.append((a, b))
        Xs = inputs.device_uniform(M, N, 3, inputs.STREAM_C, cplx, dev)
        Cout = torch.empty((M, N), dtype=tdt, device=dev)
        byts, flops = _algorithmic(op, cplx, K, M, N, 4 if f32 else 8)
        out = []
        for v in variants:
            name = codegen.variant_name(v)
            rec = dict(base or {}, op=op, dt=dt, M=M, N=N, name=name, cfg=v["cfg"], K=K)
            if name not in self.names:
                rec.update(ok=False, error="not compiled")
                out.append(rec)
                continue
            _lib.check(_lib.tsg_force_variant(name))
            try:
                acc = "f32" if codegen.is_a32(dt) else "f64"
                if op == "tsmttsm":
                    once = lambda: api.tsmttsm(Ai, Bi, acc=acc).clone()
                    call = (lambda s: api.tsmttsm(s[0], s[1], out=Cout, acc=acc))
                else:
                    once = lambda: api.tsmm(Ai, Xi, acc=acc).to(exact.dtype)
                    call = (lambda s: api.tsmm(s[0], Xs, out=s[1], acc=acc))
                ok = bool(torch.equal(once(), exact))
                _lib.check(_lib.tsg_set_grid_limit(3))
                try:
                    ok = ok and bool(torch.equal(once(), exact))
                finally:
                    _lib.tsg_set_grid_limit(0)
                for w in range(self.warmup):
                    call(sets[w % R])
                evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                       for _ in range(self.reps)]
                for i in range(self.reps):
                    evs[i][0].record()
                    call(sets[(self.warmup + i) % R])
                    evs[i][1].record()
                torch.cuda.synchronize()
                times = sorted(e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs)
                t = times[len(times) // 2]
                roof = max(byts / HBM_PEAK, flops / FP64_PEAK)
                rec.update(ok=ok, us=round(t * 1e6, 2), us_min=round(times[0] * 1e6, 2),
                           GBps=round(byts / t / 1e9, 1), GFLOPs=round(flops / t / 1e9, 1),
                           roof_frac=round(roof / t, 4))
            finally:
                _lib.tsg_force_variant(None)
            out.append(rec)
        return out


def _read_db(path, key):
    done = {}
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                try:
                    r = json.loads(line)
                    done[key(r)] = r
                except (ValueError, KeyError):
                    pass
    return done


def _show(rec):
    print("[tune] %-50s %9.1f us %7.1f GB/s roof %.3f %s" % (
        rec["name"] + ("" if "cls" not in rec else " %dx%d" % (rec["M"], rec["N"])), rec.get("us", -1),
        rec.get("GBps", 0), rec.get("roof_frac", 0), "" if rec["ok"] else rec.get("error", "MISMATCH")), flush=True)


def cmd_run(args):
    os.environ.setdefault("TSG_LIBRARY", TUNE_LIB)
    sys.path.insert(0, ROOT)
    from paper_1905_03136_amd import codegen
    timer = _Timer(args.K, args.warmup, args.reps)
    groups = {}
    for v in codegen.tuning_variants(_widths(args.widths)):
        if v["M"] == 0:
            continue
        groups.setdefault((v["op"], v["dt"], v["M"], v["N"]), []).append(v)
    done = _read_db(args.db, lambda r: r["name"])
    db = open(args.db, "a")
    t_start = time.time()
    dtypes = set(args.dtypes.split(",")) if args.dtypes else None
    ops = set(args.ops.split(",")) if args.ops else None
    for key in sorted(groups, key=lambda k: (k[0], k[1], k[2] * k[3])):
        op, dt, M, N = key
        if (dtypes and dt not in dtypes) or (ops and op not in ops):
            continue
        cands = [v for v in groups[key] if codegen.variant_name(v) not in done]
        if args.prune:
            # the performance model drops candidates predicted far slower than
            # the best prediction (register use from the tuning build's records)
            from paper_1905_03136_amd import build, model
            res = build.variant_resources(cands, tag="_" + args.prune_tag)
            kept = model.prune(cands, args.K, res, args.prune)
            print("[tune] %s %s %dx%d: model keeps %d of %d candidates" % (op, dt, M, N, len(kept), len(cands)),
                  flush=True)
            cands = kept
        for rec in timer.measure(op, dt, M, N, cands):
            db.write(json.dumps(rec) + "\n")
            db.flush()
            done[rec["name"]] = rec
            _show(rec)
    db.close()
    print("[tune] done in %.0f s" % (time.time() - t_start), flush=True)
    write_table(args.db, args.out, args.merge)


def generic_tuning_variants():
    """Every candidate of every run-time-width class of the autotuned types,
    each with the widths its configuration can compute (so that a forced
    variant never runs beyond them)."""
    from paper_1905_03136_amd import codegen
    out, seen = [], set()
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        for dt in codegen.GEN_TUNED_DTYPES:
            for cls in classes:
                for cfg in codegen.generic_candidates(op, dt, cls):
                    mx, nx = codegen.generic_capacity(op, cfg)
                    v = dict(op=op, dt=dt, M=0, N=0, maxM=mx, maxN=nx, cfg=cfg)
                    if codegen.variant_name(v) not in seen:
                        seen.add(codegen.variant_name(v))
                        out.append(v)
    return out


def cmd_generic(args):
    """GPU: time the candidates of every run-time-width class on the class's
    pairs and write the choice of each class (the fastest correct one by the
    mean over the pairs of its time over the pair's best time) into the
    table's "generic" list."""
    sys.path.insert(0, ROOT)
    from paper_1905_03136_amd import build, codegen
    os.environ.setdefault("TSG_LIBRARY", build.tagged_lib(args.tag))
    timer = _Timer(args.K, args.warmup, args.reps)
    done = _read_db(args.db, lambda r: (r["name"], r["M"], r["N"]))
    db = open(args.db, "a")
    t_start = time.time()
    ops = set(args.ops.split(",")) if args.ops else None
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        if ops and op not in ops:
            continue
        for dt in codegen.GEN_TUNED_DTYPES:
            for cls in classes:
                vs = []
                for cfg in codegen.generic_candidates(op, dt, cls):
                    mx, nx = codegen.generic_capacity(op, cfg)
                    vs.append(dict(op=op, dt=dt, M=0, N=0, maxM=mx, maxN=nx, cfg=cfg))
                for M, N in codegen.generic_pairs(op, cls):
                    todo = [v for v in vs if (codegen.variant_name(v), M, N) not in done]
                    for rec in timer.measure(op, dt, M, N, todo, base=dict(cls=list(cls))):
                        db.write(json.dumps(rec) + "\n")
                        db.flush()
                        done[(rec["name"], M, N)] = rec
                        if args.verbose or not rec["ok"]:
                            _show(rec)
                print("[tune] %s %s class %dx%d: %d candidates timed (%.0f s)" % (
                    op, dt, cls[0], cls[1], len(vs), time.time() - t_start), flush=True)
    db.close()
    write_generic(args.db, args.out)


def write_generic(db_path, out_path):
    """The "generic" list of the table from a database of class timings."""
    from paper_1905_03136_amd import codegen
    recs = {}
    with open(db_path) as f:
        for line in f:
            try:
                r = json.loads(line)
            except ValueError:
                continue
            if "cls" in r:
                recs[(r["name"], r["M"], r["N"])] = r
    entries = []
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        for dt in codegen.GEN_TUNED_DTYPES:
            for cls in classes:
                pairs = codegen.generic_pairs(op, cls)
                by = {}
                for (name, M, N), r in recs.items():
                    if r["op"] == op and r["dt"] == dt and tuple(r["cls"]) == tuple(cls):
                        by.setdefault(name, {})[(M, N)] = r
                # a candidate counts only if it is exact and timed on every pair
                full = {n: d for n, d in by.items()
                        if all(p in d and d[p].get("ok") and d[p].get("us") for p in pairs)}
                if not full:
                    continue
                best = {p: min(d[p]["us"] for d in full.values()) for p in pairs}
                score = {n: sum(d[p]["us"] / best[p] for p in pairs) / len(pairs) for n, d in full.items()}
                win = min(score, key=score.get)
                d = full[win]
                mx, nx = codegen.generic_limits(op, cls)
                e = dict(op=op, dt=dt, maxM=mx, maxN=nx, cfg=d[pairs[0]]["cfg"], name=win,
                         score=round(score[win], 4), candidates=len(full),
                         pairs=[[M, N, d[(M, N)]["us"], d[(M, N)]["roof_frac"]] for M, N in pairs])
                # the fastest configuration without layout requirements on A
                # (served to calls whose rows are not contiguous)
                if codegen.needs_layout(e["cfg"]):
                    plain = {n: sc for n, sc in score.items() if not codegen.needs_layout(full[n][pairs[0]]["cfg"])}
                    if plain:
                        pw = min(plain, key=plain.get)
                        e.update(plain_cfg=full[pw][pairs[0]]["cfg"], plain_name=pw, plain_score=round(plain[pw], 4))
                entries.append(e)
    tab = {"entries": []}
    if os.path.exists(out_path):
        with open(out_path) as f:
            tab = json.load(f)
    tab["generic"] = entries
    with open(out_path, "w") as f:
        json.dump(tab, f, indent=1)
        f.write("\n")
    print("[tune] wrote %s (%d run-time-width classes)" % (out_path, len(entries)), flush=True)


def cmd_batched(args):
    """Autotune the batched form on its workload: every (input bytes per
    slab, queue interleave) pair of the grid is timed on one persistent
    launch of the batched orthogonalisation (``inputs.batched_instances``:
    `count` instances, K_i log-uniform in [2^16, 2^22]); the fastest pair is
    written to the table's "batched" key, from which the generator compiles
    the library's defaults."""
    sys.path.insert(0, ROOT)
    import torch

    from paper_1905_03136_amd import api, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    shapes = inputs.batched_instances(args.count, seed=0)
    pairs = []
    for i, (K, M, N) in enumerate(shapes):
        V = inputs.device_uniform(K, M, 100 + i, inputs.STREAM_V0, False, dev)
        V.mul_((3.0 / K) ** 0.5)
        W = inputs.device_uniform(K, N, 100 + i, inputs.STREAM_W0, False, dev)
        pairs.append((V, W))
    byts = sum(8 * K * (2 * M + 3 * N) for K, M, N in shapes)
    db = open(args.db, "a")
    recs = []
    for ib in [int(x) for x in args.item_bytes.split(",")]:
        for lag in [int(x) for x in args.lags.split(",")]:
            os.environ["TSG_ORTH_ITEM_BYTES"] = str(ib)
            os.environ["TSG_ORTH_LAG"] = str(lag)
            plan = api.OrthPlan(pairs)
            try:
                for _ in range(args.warmup):
                    plan.launch()
                torch.cuda.synchronize()
                ts = []
                for _ in range(args.reps):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    plan.launch()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                plan.check()
            finally:
                plan.close()
            ts.sort()
            rec = dict(form="batched", count=args.count, item_bytes=ib, lag=lag, us=round(ts[len(ts) // 2] * 1e6, 1),
                       us_min=round(ts[0] * 1e6, 1), GBps=round(byts / ts[len(ts) // 2] / 1e9, 1))
            recs.append(rec)
            db.write(json.dumps(rec) + "\n")
            db.flush()
            print("[tune] batched item bytes %9d lag %3d: %8.1f us %7.1f GB/s" % (ib, lag, rec["us"], rec["GBps"]),
                  flush=True)
    db.close()
    for k in ("TSG_ORTH_ITEM_BYTES", "TSG_ORTH_LAG"):
        os.environ.pop(k, None)
    best = min(recs, key=lambda r: r["us"])
    tab = {"entries": []}
    if os.path.exists(args.out):
        with open(args.out) as f:
            tab = json.load(f)
    tab["batched"] = dict(item_bytes=best["item_bytes"], lag=best["lag"], us=best["us"], GBps=best["GBps"],
                          count=args.count, grid=[[r["item_bytes"], r["lag"], r["us"]] for r in recs])
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
        f.write("\n")
    print("[tune] batched: item bytes %d, lag %d (%.1f us); wrote %s" % (best["item_bytes"], best["lag"], best["us"],
                                                                         args.out), flush=True)


def write_table(db_path, out_path, merge=None):
    """Fastest correct configuration per (op, dtype, M, N) from the database;
    entries of an existing table ``merge`` that the database does not cover
    are kept."""
    from paper_1905_03136_amd.codegen import A32_TWIN, needs_layout
    best, plain = {}, {}
    # a binary32-arithmetic type takes the fastest of its own records and its
    # binary64-arithmetic twin's (the twin is exact in its products and wins
    # wherever it is as fast); tune both types in one run
    if merge and os.path.exists(merge):
        with open(merge) as f:
            for e in json.load(f).get("entries", []):
                key = (e["op"], e["dt"], e["M"], e["N"])
                best[key] = dict(e, _kept=True)
                if e.get("plain_cfg"):
                    plain[key] = dict(cfg=e["plain_cfg"], name=e.get("plain_name"), us=e.get("plain_us"), _kept=True)
    with open(db_path) as f:
        for line in f:
            try:
                r = json.loads(line)
            except ValueError:
                continue
            if not r.get("ok") or "us" not in r:
                continue
            keys = [(r["op"], r["dt"], r["M"], r["N"])]
            # a binary64-arithmetic kernel also serves its binary32-arithmetic twin type
            keys += [(r["op"], a, r["M"], r["N"]) for a, t in A32_TWIN.items() if t == r["dt"]]
            for key in keys:
                if key not in best or best[key].get("_kept") or r["us"] < best[key]["us"]:
                    best[key] = r
                # fastest configuration without layout requirements on A
                if not needs_layout(r["cfg"]) and (key not in plain or plain[key].get("_kept") or
                                                   r["us"] < plain[key]["us"]):
                    plain[key] = r
    entries = []
    for k, r in sorted(best.items(), key=lambda kv: (kv[0][0], kv[0][1], kv[0][2] * kv[0][3])):
        e = dict(op=k[0], dt=k[1], M=k[2], N=k[3], cfg=r["cfg"], name=r["name"], us=r["us"],
                 GBps=r["GBps"], roof_frac=r["roof_frac"], K=r["K"])
        if needs_layout(r["cfg"]) and k in plain:
            e.update(plain_cfg=plain[k]["cfg"], plain_name=plain[k]["name"], plain_us=plain[k]["us"])
        entries.append(e)
    tab = {"entries": entries}
    # the batched form's parameters and the run-time-width classes are kept
    # from the merged table
    for key in ("batched", "generic"):
        for src in (merge, out_path):
            if src and os.path.exists(src):
                with open(src) as f:
                    b = json.load(f).get(key)
                if b:
                    tab[key] = b
                    break
    with open(out_path, "w") as f:
        json.dump(tab, f, indent=1)
        f.write("\n")
    print("[tune] wrote %s (%d entries)" % (out_path, len(entries)), flush=True)


# design dimensions of a configuration, as the ablation reports them
_DIMENSIONS = {
    "mapping": lambda c: c["kind"],
    "rows in flight U": lambda c: c.get("U"),
    "ring depth NBUF": lambda c: c.get("NBUF", 2),
    "waves per block": lambda c: c.get("WPB"),
    "slab reads FL": lambda c: c.get("FL", 0),
    "vector tails TL": lambda c: c.get("TL", 0),
    "three-product form G3": lambda c: c.get("G3", 0),
    "C source (LDS 0 / global 1) CG": lambda c: c.get("CG", 0),
}


def ablation(db_paths, ops=None):
    from paper_1905_03136_amd.codegen import DTYPES
    """Cost of fixing one design dimension, from autotuner databases: for each
    (op, dtype, M, N) and each value v of a dimension, the fastest correct
    configuration with that value, as a slowdown over the fastest overall;
    reported as the geometric mean and the maximum over the widths where v
    was timed.  Later databases override earlier records of the same name."""
    recs = {}
    for path in db_paths:
        with open(path) as f:
            for line in f:
                try:
                    r = json.loads(line)
                except ValueError:
                    continue
                if r.get("ok") and r.get("us") and r.get("M") and (not ops or r["op"] in ops):
                    recs[(r["op"], r["dt"], r["M"], r["N"], r["name"])] = r
    groups = {}
    for (op, dt, M, N, _), r in recs.items():
        groups.setdefault((op, dt, M, N), []).append(r)
    out = {}
    for (op, dt, M, N), rs in groups.items():
        best = min(r["us"] for r in rs)
        for dim, get in _DIMENSIONS.items():
            by = {}
            for r in rs:
                v = get(r["cfg"])
                by[v] = min(by.get(v, float("inf")), r["us"])
            if len(by) < 2:
                continue
            for v, t in by.items():
                out.setdefault((op, "z" if DTYPES[dt][1] else "r", dim, v), []).append(t / best)
    rows = []
    for (op, kind, dim, v), xs in sorted(out.items(), key=lambda kv: [str(x) for x in kv[0]]):
        gm = math.exp(sum(math.log(x) for x in xs) / len(xs))
        rows.append((op, kind, dim, v, len(xs), gm, max(xs)))
    return rows


def heatmap(db_paths, op, dt, M, N, resources=None):
    """The tile-size cross section of the search at one width (the paper's
    tile heat map with register iso-lines, Section 5.2): for each tile of a
    wave (mapping and its block grid) and each number of rows in flight U,
    the fastest correct configuration (over the other dimensions) with its
    time and the registers its kernel uses (VGPR + AGPR, from the build's
    resource records).  Returns (tiles, Us, cells) with cells[(tile, U)] =
    (us, name, regs)."""
    recs = {}
    for path in db_paths:
        with open(path) as f:
            for line in f:
                try:
                    r = json.loads(line)
                except ValueError:
                    continue
                if (r.get("ok") and r.get("us") and r.get("op") == op and r.get("dt") == dt and r.get("M") == M
                        and r.get("N") == N):
                    recs[r["name"]] = r
    cells = {}
    for r in recs.values():
        c = r["cfg"]
        if c["kind"] in ("mfma", "a32") and op == "tsmttsm":
            tile = "%s %dx%d blocks, %d-way split" % (c["kind"], c["MB"], c["NB"], c.get("MW", 1))
        elif c["kind"] == "lds":
            tile = "lds %dx%d blocks, %dx%d waves" % (c["MB"], c["NB"], c["WM"], c["WN"])
        elif c["kind"] in ("mfma", "a32"):
            tile = "%s %d slices x %d blocks" % (c["kind"], c["MS"], c["NB"])
        elif c["kind"] == "valu":
            tile = "valu %dx%d" % (c["MX"], c["NX"])
        else:
            tile = c["kind"]
        u = c.get("U", c.get("RT", 0) // 4)
        res = (resources or {}).get(r["name"])
        regs = (res.get("vgpr", 0) + res.get("agpr", 0)) if res else None
        key = (tile, u)
        if key not in cells or r["us"] < cells[key][0]:
            cells[key] = (r["us"], r["name"], regs)
    tiles = sorted({k[0] for k in cells})
    us = sorted({k[1] for k in cells})
    return tiles, us, cells


def cmd_heatmap(args):
    from paper_1905_03136_amd import build, codegen
    M, N = (int(x) for x in args.width.split("x"))
    res = build.variant_resources([dict(op=args.op, dt=args.dt, M=M, N=N, maxM=M, maxN=N, cfg=c)
                                   for c in codegen.candidates(args.op, args.dt, M, N)], tag="_" + args.tag)
    tiles, us, cells = heatmap(args.db, args.op, args.dt, M, N, res)
    best = min(v[0] for v in cells.values())
    print("| tile of a wave \\ rows in flight (4-row steps) | " + " | ".join("U=%d" % u for u in us) + " |")
    print("|---|" + "---:|" * len(us))
    for t in tiles:
        row = []
        for u in us:
            v = cells.get((t, u))
            row.append("-" if not v else "%.2f (%s regs)" % (v[0] / best, v[2] if v[2] is not None else "?"))
        print("| %s | %s |" % (t, " | ".join(row)))
    print()
    print("Entries: time relative to the fastest configuration of %s %s %dx%d (%.1f us), and the registers "
          "(VGPR + AGPR per lane) of that kernel." % (args.op, args.dt, M, N, best))


def cmd_ablate(args):
    rows = ablation(args.db, set(args.ops.split(",")) if args.ops else None)
    print("| op | real/complex | dimension | value | widths | slowdown (geo. mean) | slowdown (max) |")
    print("|---|---|---|---|---:|---:|---:|")
    for op, kind, dim, v, n, gm, mx in rows:
        print("| %s | %s | %s | %s | %d | %.3f | %.2f |" % (op, "real" if kind == "r" else "complex", dim, v, n, gm, mx))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--widths", default="graded")
    b.add_argument("--ops", default="", help="comma-separated subset of tsmttsm,tsmm")
    b.add_argument("--dtypes", default="", help="comma-separated subset of r64,c128,r32,c64,r32a,c64a")
    b.add_argument("--kinds", default="", help="comma-separated subset of the mappings (valu,packed,mfma,a32,lds)")
    b.add_argument("--with-tuned", action="store_true", help="add each width's configuration in tuned.json")
    b.add_argument("--tag", default="", help="build _build/libtsgemm_<tag>.so apart from the default tuning library")
    b.add_argument("--generic", action="store_true", help="the candidates of the run-time-width classes")
    r = sub.add_parser("run")
    r.add_argument("--widths", default="graded")
    r.add_argument("--dtypes", default="", help="comma-separated subset of r64,c128,r32,c64,r32a,c64a")
    r.add_argument("--ops", default="", help="comma-separated subset of tsmttsm,tsmm")
    r.add_argument("--K", type=int, default=1 << 24)
    r.add_argument("--db", default="tune_db.jsonl")
    r.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    r.add_argument("--reps", type=int, default=5)
    r.add_argument("--warmup", type=int, default=2)
    r.add_argument("--merge", default="", help="keep the entries of this table the run does not cover")
    r.add_argument("--prune", type=float, default=0.0,
                   help="time only candidates the performance model predicts within this factor of the best")
    r.add_argument("--prune-tag", default="tune", help="build whose resource records the model reads")
    ab = sub.add_parser("ablate", help="cost of fixing each design dimension, from tuning databases")
    ab.add_argument("--db", action="append", required=True, help="a tuning database (repeatable; later ones win)")
    ab.add_argument("--ops", default="", help="comma-separated subset of tsmttsm,tsmm")
    hm = sub.add_parser("heatmap", help="tile x rows-in-flight cross section of the search at one width")
    hm.add_argument("--db", action="append", required=True)
    hm.add_argument("--op", default="tsmttsm")
    hm.add_argument("--dt", default="r64")
    hm.add_argument("--width", default="32x32")
    hm.add_argument("--tag", default="tune", help="build whose resource records give the register counts")
    bt = sub.add_parser("batched", help="GPU: input bytes per slab and queue interleave of the batched form")
    bt.add_argument("--count", type=int, default=64)
    bt.add_argument("--item-bytes", default="1048576,2097152,4194304,8388608,16777216")
    bt.add_argument("--lags", default="0,4,16,32")
    bt.add_argument("--reps", type=int, default=5)
    bt.add_argument("--warmup", type=int, default=2)
    bt.add_argument("--db", default="tune_batched.jsonl")
    bt.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    g = sub.add_parser("generic", help="GPU: configurations of the run-time-width classes")
    g.add_argument("--K", type=int, default=1 << 24)
    g.add_argument("--ops", default="", help="comma-separated subset of tsmttsm,tsmm")
    g.add_argument("--tag", default="generic", help="library built by 'build --generic --tag <tag>'")
    g.add_argument("--db", default="tune_generic.jsonl")
    g.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    g.add_argument("--reps", type=int, default=5)
    g.add_argument("--warmup", type=int, default=2)
    g.add_argument("--verbose", action="store_true", help="print every timing")
    g.add_argument("--table-only", action="store_true", help="only write the table from the database")
    t = sub.add_parser("table")
    t.add_argument("--db", default="tune_db.jsonl")
    t.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    t.add_argument("--merge", default="")
    a = ap.parse_args(argv)
    if a.cmd == "build":
        cmd_build(a)
    elif a.cmd == "run":
        cmd_run(a)
    elif a.cmd == "ablate":
        cmd_ablate(a)
    elif a.cmd == "batched":
        cmd_batched(a)
    elif a.cmd == "heatmap":
        cmd_heatmap(a)
    elif a.cmd == "generic":
        if a.table_only:
            write_generic(a.db, a.out)
        else:
            cmd_generic(a)
    else:
        write_table(a.db, a.out, a.merge)


if __name__ == "__main__":
    main()
