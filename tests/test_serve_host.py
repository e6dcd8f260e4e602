"""Host logic of the serving loop that needs no GPU."""
import gc

from paper_2411_01964_amd import serve


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
    assert serve.footprint(lo, hi, True) - serve.footprint(lo, hi, False) == 5000
