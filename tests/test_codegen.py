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
    v = codegen.all_variants()
    for op in codegen.OPS:
        for dt in codegen.DTYPES:
            gens = [x for x in v if x["op"] == op and x["dt"] == dt and x["M"] == 0]
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
