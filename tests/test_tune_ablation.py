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
