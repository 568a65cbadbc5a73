"""The stored oracle digests of the batched workload (tests/golden/
batch_oracle.json, written by tests/golden/make_batch_oracle.py) still match
the workload generator, the subset rule and the oracle: the subset and the
problem sizes agree, and the smallest heat and Euler problems of each
precision are re-stepped on the oracle here and hashed again."""
import batch_oracle as bo


def test_golden_matches_workload_and_oracle():
    golden = bo.load_golden()
    assert golden["steps"] == bo.STEPS
    for pair in ("f64", "f32"):
        probs, ids, hosts = bo.problems(pair)
        entry = golden["pairs"][pair]
        assert entry["subset"] == bo.subset(probs)
        rows = {r["problem"]: r for r in entry["problems"]}
        assert sorted(rows) == entry["subset"]
        for i, r in rows.items():
            assert r["n"] == probs[i].n and r["eq"] == ids[i]
            assert r["cells"] == bo.sample_cells(ids[i], probs[i].n).size
        for kind in ("heat", "euler"):
            i = min((i for i in rows if probs[i].eq == kind), key=lambda i: probs[i].n)
            cells, vals = bo.sample(ids[i], hosts[i], bo.STEPS)
            assert bo.digest(vals) == rows[i]["sha256"], (pair, kind, i)
