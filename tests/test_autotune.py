"""Autotuner cache (CPU): keys depend on every shape parameter, entries
survive a round trip through the file."""
import json

import paper_1109_6587_amd.autotune as A
from workloads import random_case


def test_key_and_cache(tmp_path):
    a = [random_case(1, 10, 10, 4.0, 1.0, 4.0, 1.0, 32, 32, 17)]
    b = [random_case(1, 10, 11, 4.0, 1.0, 4.0, 1.0, 32, 32, 17)]
    k1 = A.batch_key(a, "mixed", device="x")
    assert k1 == A.batch_key(a, "mixed", device="x")
    assert k1 != A.batch_key(b, "mixed", device="x")
    assert k1 != A.batch_key(a, "fp64", device="x")
    assert k1 != A.batch_key(a, "mixed", device="y")
    p = tmp_path / "sub" / "cache.json"
    A._store(str(p), {k1: {"branches": 2}})
    assert A._load(str(p))[k1]["branches"] == 2
    p.write_text("not json")
    assert A._load(str(p)) == {}
    assert json.loads(json.dumps(A._load(str(tmp_path / "missing.json")))) == {}
