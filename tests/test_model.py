"""Performance model of the kernels (host logic only): bandwidth against
bytes in flight follows the Table-1 measurements, predictions are positive
and bounded below by the roofline of the chip's measured rates, and pruning
always keeps the best-predicted candidate."""
import json

from paper_1905_03136_amd import codegen, model


def test_bandwidth_interpolates_table1_and_saturates():
    qs = [1 << 10, 4 << 10, 8 << 10, 16 << 10, 32 << 10, 1 << 20]
    bw = [model.bandwidth(q) for q in qs]
    assert all(b > 0 for b in bw)
    assert bw[1] == model.TABLE1[0][1] * 1e9 and abs(bw[3] - 6200e9) < 1e-3 * 6200e9
    assert bw[0] < bw[1] < bw[2] < bw[3] < bw[4]
    assert bw[-1] == model.TABLE1[-1][1] * 1e9


def test_predictions_respect_the_measured_roofline():
    K = 1 << 24
    for op in ("tsmttsm", "tsmm"):
        for dt, (M, N) in (("r64", (8, 8)), ("c128", (64, 64)), ("r64", (32, 8))):
            cands = [dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=c) for c in codegen.candidates(op, dt, M, N)]
            s = 16 if dt == "c128" else 8
            floor = s * K * (M + N) / (model.TABLE1[-2][1] * 1e9)
            for v in cands:
                t = model.predict(v, K)
                assert t >= floor * 0.99
            kept = model.prune(cands, K, keep=1.2)
            best = min(cands, key=lambda v: model.predict(v, K))
            assert best in kept and len(kept) <= len(cands)


def test_evaluate_reports_whether_the_fastest_survives(tmp_path):
    K = 1 << 24
    cands = codegen.candidates("tsmttsm", "c128", 64, 64)[:6]
    db = tmp_path / "db.jsonl"
    with open(db, "w") as f:
        for i, c in enumerate(cands):
            v = dict(op="tsmttsm", dt="c128", M=64, N=64, maxM=64, maxN=64, cfg=c)
            f.write(json.dumps(dict(op="tsmttsm", dt="c128", M=64, N=64, name=codegen.variant_name(v), cfg=c, K=K,
                                    ok=True, us=1000.0 + i)) + "\n")
    rows = model.evaluate([str(db)], keep=100.0)
    assert len(rows) == 1 and rows[0]["candidates"] == 6 and rows[0]["kept"] == 6 and rows[0]["best_kept"]
    assert rows[0]["slowdown"] == 1.0
