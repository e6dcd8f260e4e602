"""Host logic of the serving loop that needs no GPU."""
import gc

from paper_2411_01964_amd import esq, serve


def test_gc_pause_is_reference_counted():
    was = gc.isenabled()
    try:
        gc.enable()
        serve._gc_pause()
        serve._gc_pause()
        assert not gc.isenabled()
        serve._gc_resume()
        assert not gc.isenabled()      # a second server is still running
        serve._gc_resume()
        assert gc.isenabled()
        gc.disable()                   # a caller that had it off keeps it off
        serve._gc_pause()
        serve._gc_resume()
        assert not gc.isenabled()
    finally:
        (gc.enable if was else gc.disable)()


def test_footprint_counts_per_n_bytes():
    lo, hi = 1001, 1001 + 2 * 5000
    # the per-n bytes plus the 16-byte slack of their placement
    assert serve.footprint(lo, hi, True) - serve.footprint(lo, hi, False) == 5000 + 16
    assert serve.footprint(3, 1 << 31, False) > serve.footprint(3, 1 << 21, False)


def fake_batch(count, per_n):
    """A BatchResults over host byte tensors, as the device would fill them."""
    import numpy as np
    import torch
    sm = np.zeros(count, dtype=esq.SUMMARY_DTYPE)
    rc = np.zeros((count, esq.ESQ_RECORDS_CAP), dtype=esq.RECORD_DTYPE)
    for i in range(count):
        sm[i]["n0"], sm[i]["n_odd"], sm[i]["ksum"] = 101 + 2 * i, 7 + i, 9 + i
        sm[i]["hist"][1], sm[i]["kmax_seen"], sm[i]["n_records"] = 7 + i, 2, 2
        rc[i]["n"][:2], rc[i]["k"][:2] = (101 + 2 * i, 103 + 2 * i), (1, 2)
    s = torch.from_numpy(sm.view(np.uint8).copy())
    r = torch.from_numpy(rc.reshape(-1).view(np.uint8).copy())
    pn = [torch.full((7 + i,), i, dtype=torch.uint8) if per_n else None for i in range(count)]
    return esq.BatchResults(s, r, count, pn if per_n else None, check=True)


def test_batch_results_parse_on_demand_and_release():
    b = fake_batch(3, per_n=True)
    d = b.parse(2)
    assert d["n0"] == 105 and d["n_odd"] == 9 and d["hist"][1] == 9 and d["ksum"] == 11
    assert d["records"] == [(105, 1), (107, 2)] and d["record_flags"] == [0, 0]
    assert int(d["per_n"][0]) == 2
    r = serve.Request(105, 105 + 18, True, 0.0)
    r._src, r.t_done = (b, 2), 1.0
    serve._release_per_n(r)                 # before the result is read
    assert "per_n" not in r.result and r.result["n_odd"] == 9
    assert r.wait() is r.result             # done: no server needed
    r.result = None
    assert r.result is None


def test_batch_results_report_device_status():
    import pytest
    b = fake_batch(2, per_n=False)
    b.sm["status"][1] = 1
    with pytest.raises(esq.EsqError):
        esq.BatchResults.__init__(b, *_raw(b), check=True)


def _raw(b):
    import numpy as np
    import torch
    return (torch.from_numpy(b.sm.view(np.uint8).copy()),
            torch.from_numpy(b.rc.reshape(-1).view(np.uint8).copy()), b.count, None)
