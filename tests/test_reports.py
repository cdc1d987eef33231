"""Host-side report renderers (no GPU): the nonsymmetric sweep's tables and
the machine probes' tables are rendered from their JSON as measured."""
import json

import bench
from paper_1905_03136_amd import probes


def test_pair_table_places_every_fraction(tmp_path):
    rows = []
    for dt in ("D", "Z"):
        for M in (1, 4):
            for N in (1, 4, 8):
                rec = {"dtype": dt, "M": M, "N": N, "K": 16}
                for op, base in (("tsmttsm", 0.1), ("tsmm", 0.5)):
                    rec[op] = {"us": 1.0, "roof_frac": base + M / 100 + N / 1000 + (0.2 if dt == "Z" else 0.0),
                               "kernel": "k"}
                rows.append(rec)
    path = tmp_path / "pairs.jsonl"
    path.write_text("noise line\n" + "".join(json.dumps(r) + "\n" for r in rows)
                    + json.dumps({"pair_sweep_summary": {"x": 1}}) + "\n")
    text = bench.pair_table(str(path))
    assert text.count("| M \\\\ N | 1 | 4 | 8 |") == 4
    # row M = 4 of Z TSMM: 0.5 + 0.04 + N / 1000 + 0.2
    zt = text.split("**Z TSMM**")[1]
    assert "| 4 | 0.74 | 0.74 | 0.75 |" in zt
    assert '"pair_sweep_summary"' in text


def test_probe_markdown_tables():
    res = {"table1": {"%d,%d" % (o, i): 1000.0 * o + i for o in (1, 2) for i in (1, 4)},
           "mixes": {"1:1 streaming": {"GBps": 5384.2, "blocks_per_cu": 2, "loads_in_flight": 8}},
           "peaks": {"mfma_f64": {"1": 37.9, "2": 51.5}},
           "latency": {"1048576": {"cycles": 298.0, "ns": 124.1}}}
    text = probes.markdown(res)
    assert "| 2 | 2001 | 2004 |" in text
    assert "| 1:1 streaming | 5384 | 2 | 8 |" in text
    assert "| mfma_f64 | 37.9 | 51.5 |" in text
    assert "| 1 MiB | 298 | 124 |" in text


def test_reduction_table_rows(tmp_path):
    rec = {"M": 4, "N": 4, "K": 1000, "sets": 2, "kernel": "k",
           "fold": {"us": 12.0, "GBps": 1.0, "roof_frac": 0.0123, "overhead_vs_none": 0.2},
           "atomic": {"us": 15.0, "GBps": 1.0, "roof_frac": 0.01, "overhead_vs_none": 0.5},
           "none": {"us": 10.0, "GBps": 1.0, "roof_frac": 0.02}}
    path = tmp_path / "red.jsonl"
    path.write_text("x\n" + json.dumps(rec) + "\n")
    text = bench.reduction_table(str(path))
    assert "| 4 | 1000 | 12.0 | +20% | 15.0 | +50% | 10.0 | 0.012 |" in text


def test_vendor_table_rows(tmp_path):
    rec = {"dtype": "D", "M": 8, "N": 8, "K": 16,
           "tsmttsm": {"us": 10.0, "roof_frac": 0.8, "kernel": "k", "vendor_us": 1000.0, "vendor_roof_frac": 0.008,
                       "speedup_vs_vendor": 100.0},
           "tsmm": {"us": 20.0, "roof_frac": 0.6, "kernel": "k", "vendor_us": 40.0, "vendor_roof_frac": 0.3,
                    "speedup_vs_vendor": 2.0}}
    path = tmp_path / "v.jsonl"
    path.write_text(json.dumps(rec) + "\n" + json.dumps({"all_widths_summary": {"D_tsmttsm": {"mean": 0.8}}}) + "\n")
    text = bench.vendor_table(str(path))
    assert "| D | 8 | 10.0 | 1000.0 | 100 | 20.0 | 40.0 | 2.00 | 0.800 / 0.600 | 0.0080 / 0.300 |" in text
    assert "all_widths_summary" in text
