"""The autotuner's ablation summary on a small synthetic database (CPU)."""
import json

from paper_1905_03136_amd import tune


def test_ablation_slowdowns(tmp_path):
    db = tmp_path / "db.jsonl"
    recs = [
        # width 8: the fastest has U = 2; fixing U = 1 costs 1.5x, U = 4 costs 2x
        dict(op="tsmm", dt="r64", M=8, N=8, name="a", cfg=dict(kind="mfma", U=2, WPB=4), ok=True, us=10.0),
        dict(op="tsmm", dt="r64", M=8, N=8, name="b", cfg=dict(kind="mfma", U=1, WPB=4), ok=True, us=15.0),
        dict(op="tsmm", dt="r64", M=8, N=8, name="c", cfg=dict(kind="mfma", U=4, WPB=8), ok=True, us=20.0),
        # a wrong result never counts
        dict(op="tsmm", dt="r64", M=8, N=8, name="d", cfg=dict(kind="mfma", U=1, WPB=8), ok=False, us=1.0),
        # width 16: U = 1 is the fastest; U = 2 costs 4x
        dict(op="tsmm", dt="r64", M=16, N=16, name="e", cfg=dict(kind="mfma", U=1, WPB=4), ok=True, us=5.0),
        dict(op="tsmm", dt="r64", M=16, N=16, name="f", cfg=dict(kind="mfma", U=2, WPB=4), ok=True, us=20.0),
    ]
    db.write_text("".join(json.dumps(r) + "\n" for r in recs))
    # a later database overrides a record of the same name
    db2 = tmp_path / "db2.jsonl"
    db2.write_text(json.dumps(dict(recs[1], us=30.0)) + "\n")
    rows = {(r[2], r[3]): r for r in tune.ablation([str(db), str(db2)])}
    op, kind, dim, v, n, gm, mx = rows[("rows in flight U", 1)]
    assert (op, kind, n) == ("tsmm", "r", 2)
    assert abs(gm - (3.0 * 1.0) ** 0.5) < 1e-12 and mx == 3.0
    _, _, _, _, n, gm, mx = rows[("rows in flight U", 2)]
    assert n == 2 and abs(gm - 2.0) < 1e-12 and mx == 4.0
    _, _, _, _, n, gm, mx = rows[("rows in flight U", 4)]
    assert n == 1 and gm == 2.0
    # waves per block has two values only at width 8
    _, _, _, _, n, gm, mx = rows[("waves per block", 8)]
    assert n == 1 and gm == 2.0
    assert ("mapping", "mfma") not in rows      # one value only: no ablation


def test_runtime_width_choice(tmp_path):
    """The run-time-width class choice: the lowest mean of time over the
    pair's best time, among candidates exact and timed on every pair; the
    table's other keys are kept and a write_table run keeps the choice."""
    from paper_1905_03136_amd import codegen
    op, dt, cls = "tsmttsm", "r64", (3, 4)
    pairs = codegen.generic_pairs(op, cls)
    cands = codegen.generic_candidates(op, dt, cls)[:3]
    names = ["x", "y", "z"]
    # x: 1.0, 1.5, 1.0 of the best (mean 1.167); y: 1.2, 1.0, 1.2 (mean 1.133);
    # z: fastest everywhere but wrong on one pair
    ratio = {"x": (1.0, 1.5, 1.0), "y": (1.2, 1.0, 1.2), "z": (0.5, 0.5, 0.5)}
    recs = []
    for nm, cfg in zip(names, cands):
        for i, (M, N) in enumerate(pairs):
            recs.append(dict(op=op, dt=dt, M=M, N=N, name=nm, cfg=cfg, K=1, cls=list(cls), ok=not (nm == "z" and i == 1),
                             us=100.0 * ratio[nm][i], roof_frac=0.5, GBps=1.0))
    # a candidate missing a pair does not count
    recs.append(dict(recs[0], name="w", us=1.0))
    db = tmp_path / "gen.jsonl"
    db.write_text("".join(json.dumps(r) + "\n" for r in recs))
    out = tmp_path / "tuned.json"
    out.write_text(json.dumps({"entries": [], "batched": {"item_bytes": 1, "lag": 0}}))
    tune.write_generic(str(db), str(out))
    tab = json.loads(out.read_text())
    assert tab["batched"] == {"item_bytes": 1, "lag": 0}
    (e,) = tab["generic"]
    assert (e["op"], e["dt"], e["maxM"], e["maxN"]) == (op, dt) + codegen.generic_limits(op, cls)
    assert e["name"] == "y" and e["cfg"] == cands[1] and e["candidates"] == 2
    assert abs(e["score"] - (1.2 / 1.0 + 1.0 / 1.0 + 1.2 / 1.0) / 3) < 1e-4
    # the exact-width table writer keeps the run-time-width choice
    tdb = tmp_path / "db.jsonl"
    tdb.write_text(json.dumps(dict(op="tsmm", dt="r64", M=8, N=8, name="a", cfg=dict(kind="mfma", MS=2, NB=1, U=2,
                                                                                           WPB=4),
                                   ok=True, us=10.0, GBps=1.0, roof_frac=0.5, K=1)) + "\n")
    tune.write_table(str(tdb), str(out))
    tab = json.loads(out.read_text())
    assert tab["generic"][0]["name"] == "y" and len(tab["entries"]) == 1
