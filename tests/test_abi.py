"""The C-ABI library loads on a machine without a GPU and exports every
function that include/esq.h declares; struct layouts agree with the header.
No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2411_01964_amd import esq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = esq.lib()
    names = declared_functions()
    assert names, "no declarations parsed"
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(esq.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "esq.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(esq_summary), sizeof(esq_record),'
        ' offsetof(esq_summary, ksum), offsetof(esq_summary, status), offsetof(esq_record, k),'
        ' offsetof(esq_record, flags));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(esq.Summary), ctypes.sizeof(esq.Record),
                   esq.Summary.ksum.offset, esq.Summary.status.offset, esq.Record.k.offset,
                   esq.Record.flags.offset]


def test_calls_before_init_fail_cleanly():
    L = esq.lib()
    L.esq_shutdown()
    rc = L.esq_verify_range(3, 100, 0, None, None, None, None, 0, None)
    assert rc == -5  # ESQ_ENOINIT
    assert b"esq_init" in L.esq_last_error()
    rc = L.esq_sieve_segment(1, 100, None, None)
    assert rc == -5
    assert L.esq_verify_range_noalloc(3, 100, 0, None, None, None, None, 0, None) == -5
    lo = (ctypes.c_uint64 * 1)(3)
    hi = (ctypes.c_uint64 * 1)(1001)
    out = ctypes.c_uint64(7)
    assert L.esq_scratch_bytes(1, lo, hi, 0, ctypes.byref(out)) == -5
    assert L.esq_scratch_bytes(1, lo, hi, 0, None) == -1   # ESQ_EINVAL


def test_measurement_calls_validate_arguments():
    L = esq.lib()
    assert L.esq_phase_take(None) == -1          # ESQ_EINVAL
    assert L.esq_measure_ceilings(None) == -1
    L.esq_shutdown()
    out = (ctypes.c_uint64 * 3)()
    assert L.esq_phase_take(out) == -5           # ESQ_ENOINIT
    for name, bad in (("sieve_seg_log2", 9), ("sieve_seg_log2", 21), ("phase_clock", 2)):
        with pytest.raises(esq.EsqError):
            esq.set_param(name, bad)
    assert esq.get_param("sieve_seg_log2") == 20 and esq.get_param("phase_clock") == 0


def test_param_validation():
    assert esq.get_param("seg_log2") >= 10
    with pytest.raises(esq.EsqError):
        esq.set_param("seg_log2", 25)
    with pytest.raises(esq.EsqError):
        esq.set_param("kh", 0)
    for name in ("block", "per_n_block", "sieve_block"):
        for bad in (0, 100, 2048):
            with pytest.raises(esq.EsqError):
                esq.set_param(name, bad)
    assert (esq.get_param("block"), esq.get_param("per_n_block"), esq.get_param("sieve_block")) == (512, 1024, 1024)
    with pytest.raises(esq.EsqError):
        esq.set_param("no_such_knob", 1)
    assert esq.get_param("no_such_knob") == -1
    old = esq.get_param("kh")
    esq.set_param("kh", 7)
    assert esq.get_param("kh") == 7
    esq.set_param("kh", old)


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2411_01964_amd", "esq.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")


def test_numpy_views_match_header_layout():
    import numpy as np
    assert esq.SUMMARY_DTYPE.itemsize == ctypes.sizeof(esq.Summary)
    assert esq.SUMMARY_DTYPE.fields["ksum"][1] == esq.Summary.ksum.offset
    assert esq.SUMMARY_DTYPE.fields["status"][1] == esq.Summary.status.offset
    assert esq.RECORD_DTYPE.fields["k"][1] == esq.Record.k.offset
    # a summary written through ctypes reads back through the numpy view
    s = esq.Summary()
    s.n0, s.n_odd, s.ksum, s.kmax_seen, s.n_records, s.status = 3, 7, 11, 5, 2, 1
    s.hist[4] = 9
    v = np.frombuffer(bytes(s), dtype=esq.SUMMARY_DTYPE)[0]
    assert (v["n0"], v["n_odd"], v["ksum"], v["kmax_seen"], v["n_records"], v["status"]) == (3, 7, 11, 5, 2, 1)
    assert v["hist"][4] == 9
