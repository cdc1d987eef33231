"""Host logic of the code generator: deterministic output, a variant for
every width pair, unique names."""
import itertools

from paper_1905_03136_amd import codegen


def test_emission_is_deterministic(tmp_path):
    v = codegen.all_variants()
    f1 = codegen.emit(str(tmp_path / "a"), v)
    f2 = codegen.emit(str(tmp_path / "b"), v)
    for a, b in zip(f1, f2):
        assert open(a).read() == open(b).read()


def test_every_width_pair_is_served():
    """Every (M, N) has a run-time-width variant; the binary32-arithmetic types
    use their binary64-arithmetic twin's (the runtime falls back to them)."""
    v = codegen.all_variants()
    for op in codegen.OPS:
        for dt in codegen.DTYPES:
            served = codegen.A32_TWIN.get(dt, dt)
            gens = [x for x in v if x["op"] == op and x["dt"] == served and x["M"] == 0]
            for M, N in itertools.product(range(1, 65), repeat=2):
                assert any(M <= g["maxM"] and N <= g["maxN"] for g in gens), (op, dt, M, N)


def test_names_unique_and_graded_widths_exact():
    v = codegen.all_variants(codegen.GRADED + codegen.SQUARE_ALL)
    names = [codegen.variant_name(x) for x in v]
    assert len(names) == len(set(names))
    exact = {(x["op"], x["dt"], x["M"], x["N"]) for x in v if x["M"]}
    for op in codegen.OPS:
        for dt in codegen.DTYPES:
            widths = codegen.PRECISION if codegen.is_f32(dt) else codegen.GRADED + codegen.SQUARE_ALL
            for M, N in widths:
                assert (op, dt, M, N) in exact


def test_binary32_storage_uses_matrix_core_kinds_only():
    for op in codegen.OPS:
        for dt in codegen.F32_DTYPES:
            for M, N in codegen.PRECISION + [(3, 3), (40, 5)]:
                assert all(c["kind"] != "valu" and not c.get("VA") for c in codegen.candidates(op, dt, M, N))
                assert codegen.default_config(op, dt, M, N)["kind"] != "valu"
    assert all(v["cfg"]["kind"] != "valu" for v in codegen.generic_variants() if codegen.is_f32(v["dt"]))


def test_default_configs_respect_register_budget():
    for op in codegen.OPS:
        for dt, (_, cplx) in codegen.DTYPES.items():
            cw = 2 if cplx else 1
            for w in range(1, 65):
                c = codegen.default_config(op, dt, w, w)
                if c["kind"] == "valu" and op == "tsmttsm":
                    assert w * w * cw + 2 * c["U"] * 2 * w * cw <= 100
                if c["kind"] == "mfma" and op == "tsmttsm":
                    assert c["MB"] * c["NB"] * 4 * cw <= 64


def test_binary32_arithmetic_candidates_and_defaults():
    """r32a / c64a: their own binary32-product kernels (register rings, and
    for TSMTTSM the LDS-staged kernel) plus every candidate of the
    binary64-arithmetic twin (which has no LDS-staged kernel for binary32
    storage); the tuning library holds only their own."""
    for op in codegen.OPS:
        for dt, twin in codegen.A32_TWIN.items():
            for M, N in ((32, 32), (64, 64), (8, 32)):
                c = codegen.candidates(op, dt, M, N)
                own = [x for x in c if x["kind"] in ("a32", "lds")]
                assert own and len(c) == len(own) + len(codegen.candidates(op, twin, M, N))
                assert any(x["kind"] == "lds" for x in own) == (op == "tsmttsm" and max(M, N) > 16)
                assert codegen.default_config(op, dt, M, N)["kind"] == "a32"
    tv = codegen.tuning_variants([(32, 32)])
    assert all(x["cfg"]["kind"] in ("a32", "lds") for x in tv if x["M"] and codegen.is_a32(x["dt"]))
    names = {codegen.variant_name(x) for x in tv}
    assert "tsmttsm_r32a_32x32_a32_b2x2w1_u2" in names


def test_batched_parameters_reach_the_generated_table(tmp_path):
    """The autotuner's batched-form choice (tuned.json key "batched") is
    compiled into the generated registry table; without it the defaults are."""
    import json
    tab = tmp_path / "tuned.json"
    tab.write_text(json.dumps({"entries": [], "batched": {"item_bytes": 8388608, "lag": 16, "us": 1.0}}))
    b = codegen.tuned_batched(str(tab))
    assert b == {"item_bytes": 8388608, "lag": 16}
    assert codegen.tuned_batched(str(tmp_path / "missing.json")) == codegen.ORTH_DEFAULTS
    files = codegen.emit(str(tmp_path / "gen"), [], batched=b)
    text = open([f for f in files if f.endswith("tsg_table.hip")][0]).read()
    assert "const int64_t kOrthItemBytes = 8388608;" in text and "const int kOrthLag = 16;" in text


def _first_cover(gens, M, N):
    for g in gens:
        if M <= g["maxM"] and N <= g["maxN"]:
            return g
    return None


def test_runtime_width_classes_listed_before_their_containers():
    """A class precedes every class that contains it, so the first record
    covering (M, N) is the tightest class."""
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        for i, a in enumerate(classes):
            for b in classes[:i]:
                assert not (a[0] <= b[0] and a[1] <= b[1]), (op, a, b)


def test_runtime_width_pairs_lie_in_their_class():
    """The pairs a class is tuned on are non-square and run on that class."""
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        for cls in classes:
            lims = [codegen.generic_limits(op, c) for c in classes]
            for M, N in codegen.generic_pairs(op, cls):
                assert M != N
                first = next(i for i, (mx, nx) in enumerate(lims) if M <= mx and N <= nx)
                assert classes[first] == cls, (op, cls, M, N)


def test_runtime_width_candidates_compute_their_class(tmp_path):
    """Every candidate of a class, and whatever the table picks, computes at
    least the widths the class serves (a forced or chosen kernel never runs
    beyond its blocks); a synthetic table's choices are the ones emitted."""
    import json
    entries = []
    for op, classes in (("tsmttsm", codegen.GEN_TSMTTSM_CLASSES), ("tsmm", codegen.GEN_TSMM_CLASSES)):
        for dt in codegen.GEN_TUNED_DTYPES:
            for cls in classes:
                mx, nx = codegen.generic_limits(op, cls)
                cands = codegen.generic_candidates(op, dt, cls)
                assert cands, (op, dt, cls)
                for c in cands:
                    cm, cn = codegen.generic_capacity(op, c)
                    assert cm >= mx and cn >= nx, (op, dt, cls, c)
                entries.append(dict(op=op, dt=dt, maxM=mx, maxN=nx, cfg=cands[-1]))
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps({"entries": [], "generic": entries}))
    gens = codegen.generic_variants(str(path))
    for op in codegen.OPS:
        for dt in codegen.GEN_TUNED_DTYPES:
            mine = [g for g in gens if g["op"] == op and g["dt"] == dt and not g["cfg"].get("RB")]
            for M, N in itertools.product(range(1, 65), repeat=2):
                g = _first_cover(mine, M, N)
                assert g is not None, (op, dt, M, N)
                if g["cfg"]["kind"] == "mfma":
                    cm, cn = codegen.generic_capacity(op, g["cfg"])
                    assert M <= cm and N <= cn
            for cls in (codegen.GEN_TSMTTSM_CLASSES if op == "tsmttsm" else codegen.GEN_TSMM_CLASSES):
                mx, nx = codegen.generic_limits(op, cls)
                want = [e["cfg"] for e in entries if (e["op"], e["dt"], e["maxM"], e["maxN"]) == (op, dt, mx, nx)]
                got = [g["cfg"] for g in mine if (g["maxM"], g["maxN"]) == (mx, nx)]
                assert got[:1] == want, (op, dt, cls)
                # a kernel with layout requirements is followed by one without
                assert not codegen.needs_layout(got[-1]), (op, dt, cls)


def test_product_runtime_width_variants_fit_their_kernels():
    """In the shipped table every run-time-width record's widths lie within
    what its kernel computes (and the beta != 0 twins within theirs)."""
    for g in codegen.generic_variants():
        if g["cfg"]["kind"] == "mfma":
            cm, cn = codegen.generic_capacity(g["op"], g["cfg"])
            assert g["maxM"] <= cm and g["maxN"] <= cn, codegen.variant_name(g)


def test_layout_restricted_kernels_have_a_fallback_and_flags():
    """Kernels that need contiguous rows or 16-byte alignment (slab reads,
    LDS staging, the dot product) carry those flags in their registry record
    and are followed by a kernel without the need: of the same width, or a
    run-time-width one covering it (the shipped table's choices)."""
    import os
    v = codegen.all_variants(None, os.path.join(os.path.dirname(codegen.__file__), "tuned.json"))
    by, gens = {}, []
    for x in v:
        if x["M"]:
            by.setdefault((x["op"], x["dt"], x["M"], x["N"]), []).append(x)
        elif not codegen.needs_layout(x["cfg"]) and not x["cfg"].get("RB"):
            gens.append(x)

    def generic_covers(op, dt, M, N):
        dt = codegen.A32_TWIN.get(dt, dt)
        return any(g["op"] == op and g["dt"] == dt and M <= g["maxM"] and N <= g["maxN"] for g in gens)
    seen = set()
    for key, xs in by.items():
        for i, x in enumerate(xs):
            c = x["cfg"]
            if not codegen.needs_layout(c):
                continue
            seen.add(c["kind"])
            rec = codegen._record(x, "launch_x")
            fields = [f.strip() for f in rec.split("{")[1].split("}")[0].split(",")]
            flat_a, align16 = int(fields[12]), int(fields[14])
            if c["kind"] in ("lds", "dot"):
                assert flat_a == 1 and align16 == 1, codegen.variant_name(x)
            assert (any(not codegen.needs_layout(y["cfg"]) and not y["cfg"].get("RB") for y in xs[i + 1:])
                    or generic_covers(*key)), codegen.variant_name(x)
    assert {"lds", "dot"} <= seen
