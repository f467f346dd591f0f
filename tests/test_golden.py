"""The stored oracle record (tests/golden/tiny_oracle.json, written by
tests/golden/make_golden.py from oracle/ only) is reproduced by the oracle as
it stands: any change to the oracle's arithmetic shows here and has to be
justified and the record rewritten by the script."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden  # noqa: E402


def test_oracle_reproduces_the_golden_record():
    with open(os.path.join(HERE, "golden", "tiny_oracle.json")) as fh:
        rec = json.load(fh)
    now = make_golden.compute()
    assert set(now) == set(rec)
    for key, val in rec.items():
        if key in ("model", "seeds", "states"):
            assert now[key] == val
            continue
        a, b = np.asarray(now[key], dtype=float), np.asarray(val, dtype=float)
        assert a.shape == b.shape, key
        scale = max(float(np.abs(b).max()), 1e-300)
        assert float(np.abs(a - b).max()) <= 1e-12 * scale, key
