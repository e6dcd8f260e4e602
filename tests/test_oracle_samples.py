"""The stored oracle samples that the full-size GPU parity tests compare
against (written by tests/golden/make_oracle_samples.py, which calls only
the oracle): the seeded generator still draws the stored n, the stored
aggregates agree with the stored least k, and seeded spot checks of the
stored least k agree with the oracle run here."""
import numpy as np
import pytest

import oracle
from tests.conftest import load_oracle_sample

NAMES = ["cfg2_random", "cfg2_windows", "cfg3_random", "cfg3_windows", "cfg4_sample",
         "cfg5_sample"]


def records_of(ks, ns):
    """Strict prefix maxima of the depth (an exception, k = 0, deeper than
    any k; nothing after it is a record)."""
    out, best = [], -1
    for n, k in zip(ns, ks):
        d = 1 << 30 if k == 0 else int(k)
        if d > best:
            out.append((int(n), int(k)))
            best = d
            if k == 0:
                break
    return out


@pytest.mark.parametrize("name", NAMES)
def test_stored_sample_is_consistent_and_matches_the_oracle(name):
    meta, ns, k, parts = load_oracle_sample(name)
    assert meta["n_count"] == ns.size == k.size
    assert np.bincount(k, minlength=65).tolist() == meta["hist"]
    assert np.all(ns % 2 == 1) and np.all(k >= 1)       # no exception below 2^50
    for f in meta.get("full", []):
        a, b = f["lo"], f["hi"]
        seg = next(p for p in parts if p[0] == a and p[1] == b)
        kk, nn = k[seg[2]:seg[3]], ns[seg[2]:seg[3]]
        assert np.array_equal(nn, np.arange(max(a, 3) | 1, b, 2, dtype=np.uint64))
        assert np.bincount(kk, minlength=65).tolist() == f["hist"]
        assert f["ksum"] == int(kk.astype(np.int64).sum()) and f["kmax_seen"] == int(kk.max())
        assert [tuple(x) for x in f["records"]] == records_of(kk, nn)
    rng = np.random.Generator(np.random.PCG64(97))
    pick = rng.choice(ns.size, size=24, replace=False)
    assert np.array_equal(oracle.mink_many(ns[pick]), k[pick])
