"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, element
by element on the same seeded inputs; exact equality everywhere (integer
work).  Sizes here span several segments and a ragged tail; the full-size
configurations are in test_gpu_fullsize.py."""
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_2411_01964_amd import esq, workloads
from tests.conftest import read_golden

pytestmark = pytest.mark.gpu

MAX_HI = (1 << 50) + (1 << 33)
DEFAULTS = dict(seg_log2=18, sieve_seg_log2=20, kh=13, block=512, per_n_block=1024, sieve_block=1024,
                entry_hits=12, tail_cap=1 << 20, medium_max=4095, bucket_cap=0, items_per_wg=4, stagger=72,
                priority=1, runs_per_wg=1)


@pytest.fixture(scope="module", autouse=True)
def lib_ready():
    esq.init(0, MAX_HI)
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)
    yield
    for k, v in DEFAULTS.items():
        esq.set_param(k, v)


def knobs(**kw):
    """Set the knobs in kw, the rest to their defaults; a block size given
    alone applies to the per-n mode too."""
    if "block" in kw:
        kw.setdefault("per_n_block", kw["block"])
    for k, v in DEFAULTS.items():
        esq.set_param(k, kw.get(k, v))


def words_np(t):
    return t.cpu().numpy().view(np.uint64)


def assert_same(g, o, per_n=True):
    assert g["n0"] == o["n0"] and g["n_odd"] == o["n_odd"]
    assert g["hist"] == o["hist"]
    assert g["ksum"] == o["ksum"]
    assert g["kmax_seen"] == o["kmax_seen"]
    assert g["records"] == o["records"]
    assert g["record_flags"] == o["record_flags"]
    assert g["n_records"] == o["n_records"]
    assert g["n_exceptions"] == o["n_exceptions"]
    if "exceptions" in g and g["exceptions"]:
        assert g["exceptions"] == o["exceptions"][:len(g["exceptions"])]
    if per_n:
        assert np.array_equal(g["per_n"].cpu().numpy(), o["per_n"])


# ------------------------------------------------------ Algorithm 1 alone

@pytest.mark.parametrize("lo,hi", [
    (0, 2), (1, 2), (1, 3), (2, 10), (8, 20), (25, 26), (1, 201),
    (1, 1 << 16), (7, (1 << 16) + 3), (12345, 12345 + 100003),
    ((1 << 30) + 1, (1 << 30) + 200001),
])
@pytest.mark.parametrize("seg_log2,block", [(10, 1024), (18, 256), (19, 1024), (20, 1024), (20, 64)])
def test_sieve_bits_exact(lo, hi, seg_log2, block):
    knobs(sieve_seg_log2=seg_log2, sieve_block=block)
    m0, n, w = esq.sieve_segment(lo, hi)
    om0, on, ow = oracle.sieve_bits(lo, hi)
    assert (m0 if n else om0, n) == (om0, on)
    if n:
        assert np.array_equal(words_np(w), ow)


@pytest.mark.parametrize("kw", [
    dict(sieve_seg_log2=20, sieve_block=1024, medium_max=11000),
    dict(sieve_seg_log2=20, sieve_block=128), dict(sieve_seg_log2=14, sieve_block=384),
    dict(sieve_seg_log2=19, sieve_block=1024, bucket_cap=1), dict(sieve_seg_log2=20, priority=0),
])
def test_sieve_role_split_knobs(kw):
    """Sieve alone with the loader/storer split at several block sizes (2 to
    16 waves; 384 threads: three loader and three storer waves), the largest
    medium range, and overflowing hit slots, against the oracle: a window
    above 2^32 of 3 segments of 2^20 plus a ragged tail, at an odd start
    (shifted output).  The single-role loop (64 threads) is in
    test_sieve_bits_exact."""
    knobs(**kw)
    lo = (1 << 32) + 12345
    hi = lo + 2 * 3 * (1 << 20) + 2 * 777 + 1
    m0, n, w = esq.sieve_segment(lo, hi)
    om0, on, ow = oracle_sieve_cached(lo, hi)
    assert (m0, n) == (om0, on)
    assert np.array_equal(words_np(w), ow)


@functools.lru_cache(maxsize=4)
def oracle_sieve_cached(lo, hi):
    return oracle.sieve_bits(lo, hi)


def test_sieve_at_2pow40_exact_and_moebius():
    lo, hi = (1 << 40) + 3, (1 << 40) + 3 + (1 << 22)
    knobs(sieve_seg_log2=16)
    m0, n, w = esq.sieve_segment(lo, hi)
    om0, on, ow = oracle.sieve_bits(lo, hi)
    assert (m0, n) == (om0, on)
    assert np.array_equal(words_np(w), ow)


# ------------------------------------------------------ Algorithm 2

def test_config1_full_exact():
    lo, hi = workloads.CONFIGS["odd_below_2pow22"]
    g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=64)
    o = oracle.verify_range(lo, hi, per_n=True)
    assert_same(g, o)
    assert g["n_odd"] == 2097151 and g["n_exceptions"] == 0
    assert g["records"] == [(3, 1), (11, 2), (29, 3), (533, 4), (849, 5), (434977, 6)]


@pytest.mark.parametrize("kw", [
    dict(seg_log2=10), dict(seg_log2=12, block=64), dict(seg_log2=20, block=1024),
    dict(kh=1), dict(kh=2), dict(kh=4), dict(kh=6), dict(kh=7), dict(kh=8),
    dict(entry_hits=1), dict(entry_hits=4096), dict(seg_log2=11, kh=9, block=128),
    dict(medium_max=11), dict(medium_max=11000), dict(medium_max=101, bucket_cap=1),
    dict(block=256, medium_max=8191), dict(seg_log2=16, block=128),
    dict(stagger=0, priority=0), dict(stagger=4096, priority=0), dict(stagger=0, runs_per_wg=7),
])
def test_knob_invariance(kw):
    knobs(**kw)
    lo, hi = 1, (1 << 19) + 7
    g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=64)
    o = oracle.verify_range(lo, hi, per_n=True)
    assert_same(g, o)


@pytest.mark.parametrize("lo,hi", [
    (0, 4), (3, 5), (4, 5), (5, 6), (0, 3), (3, 3), (1, 130), (127, 129),
    (1001, 1003), (2, 70), (64, 192), (129, 4099), (8191, 8195),
])
def test_edge_ranges(lo, hi):
    knobs(seg_log2=10)
    g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=64)
    o = oracle.verify_range(lo, hi, per_n=True)
    assert_same(g, o)


@pytest.mark.parametrize("kmax", [1, 2, 3, 5, 12])
def test_kmax_truncation_and_exceptions(kmax):
    knobs()
    lo, hi = 3, 1 << 20
    g = esq.verify_range(lo, hi, kmax=kmax, per_n=True, exceptions_cap=esq.ESQ_EXCEPTIONS_CAP_MAX)
    o = oracle.verify_range(lo, hi, kmax=kmax, per_n=True, exc_cap=1 << 20)
    assert_same(g, o)
    assert len(g["exceptions"]) == min(o["n_exceptions"], esq.ESQ_EXCEPTIONS_CAP_MAX)
    assert g["exceptions"] == o["exceptions"][:esq.ESQ_EXCEPTIONS_CAP_MAX]


@pytest.mark.parametrize("base,count,width,seed", [
    (1 << 40, 3, 1 << 12, 40),
    (1 << 50, 1, 1 << 11, 50),
    (1 << 33, 4, 1 << 13, 33),
])
def test_random_windows(base, count, width, seed):
    knobs()
    for lo, hi in workloads.random_windows(seed, count, width, base // 2, base):
        g = esq.verify_range(lo, hi, per_n=True)
        o = oracle.verify_range(lo, hi, per_n=True)
        assert_same(g, o)


def test_deep_path_crt_construction():
    """Remark of Section 2: n = 2^k (mod p_(k+1)^2), k = 1..7, forces least
    k >= 8; with kh = 4 those n go through the exact tail pass."""
    import sympy
    odd_primes = [3, 5, 7, 11, 13, 17, 19]
    mods = [p * p for p in odd_primes] + [2]
    res = [(1 << k) % (p * p) for k, p in zip(range(1, 8), odd_primes)] + [1]
    n, M = sympy.ntheory.modular.crt(mods, res)
    n, M = int(n), int(M)
    for kh in (4, 13):
        knobs(kh=kh)
        for t in (3, 11):
            c = n + t * M
            lo, hi = c - 600, c + 601
            g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=16)
            o = oracle.verify_range(lo, hi, per_n=True)
            assert_same(g, o)
            assert g["per_n"].cpu().numpy()[(c - g["n0"]) // 2] >= 8


def test_per_n_every_alignment():
    """Per-n bytes of one interval against the oracle, then of the same
    interval started j odd numbers later (every start mod 16, and a few
    more), against the first one shifted by j; with one and with eight waves
    per workgroup.  (The binding places each output so that its runs start
    16-byte aligned; the next test covers every other alignment.)"""
    lo, hi = (1 << 40) + 1, (1 << 40) + 1 + (1 << 22)
    knobs()
    base = esq.verify_range(lo, hi, per_n=True)
    assert_same(base, oracle.verify_range(lo, hi, per_n=True))
    ref = base["per_n"]
    for block in (512, 64):
        knobs(block=block)
        for j in list(range(0, 17)) + [63, 64, 65, 1000, 4097, 262143]:
            g = esq.verify_range(lo + 2 * j, hi, per_n=True)
            assert torch.equal(g["per_n"], ref[j:]), (block, j)
            counts = torch.bincount(ref[j:].to(torch.int64), minlength=65).cpu().tolist()
            assert g["hist"][1:] == counts[1:len(g["hist"])], (block, j)
    knobs()


def test_per_n_unaligned_output_pointer():
    """The per-n buffer given through the C-ABI at every byte offset mod 16
    (the output alignment then comes from the pointer, not from lo): same
    bytes as the aligned call, and nothing written outside the n_odd bytes."""
    import ctypes
    knobs()
    lo, hi = (1 << 44) + 1, (1 << 44) + 1 + (1 << 21)
    ref = esq.verify_range(lo, hi, per_n=True)["per_n"]
    n = ref.numel()
    lib = esq.lib()
    summary = torch.empty(esq.SUMMARY_BYTES, dtype=torch.uint8, device="cuda")
    records = torch.empty(esq.ESQ_RECORDS_CAP * esq.RECORD_BYTES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for off in range(16):
        buf = torch.full((n + 64,), 0xAB, dtype=torch.uint8, device="cuda")
        rc = lib.esq_verify_range(lo, hi, 0, ctypes.c_void_p(buf.data_ptr() + 32 + off),
                                  ctypes.c_void_p(summary.data_ptr()), ctypes.c_void_p(records.data_ptr()),
                                  None, 0, ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0, off
        torch.cuda.synchronize()
        assert torch.equal(buf[32 + off:32 + off + n], ref), off
        assert bool((buf[:32 + off] == 0xAB).all()) and bool((buf[32 + off + n:] == 0xAB).all()), off


def test_split_merge_invariance():
    knobs()
    lo, hi = (1 << 36) + 1, (1 << 36) + (1 << 22)
    whole = esq.verify_range(lo, hi)
    rng = np.random.default_rng(7)
    for mid in [lo + 2 * int(rng.integers(1, (hi - lo) // 2)) for _ in range(2)] + [lo + 8192 + 1]:
        a = esq.verify_range(lo, mid)
        b = esq.verify_range(mid, hi)
        assert [x + y for x, y in zip(a["hist"], b["hist"])] == whole["hist"]
        merged, best = [], 0
        for rn, rk in a["records"] + b["records"]:
            d = rk if rk else 1000
            if d > best:
                merged.append((rn, rk))
                best = d
        assert merged == whole["records"]


def test_repeated_runs_are_identical():
    knobs()
    lo, hi = (1 << 44) + 1, (1 << 44) + (1 << 24)
    a = esq.verify_range(lo, hi, per_n=True)
    b = esq.verify_range(lo, hi, per_n=True)
    assert a["hist"] == b["hist"] and a["records"] == b["records"]
    assert torch.equal(a["per_n"], b["per_n"])


def test_table3_windows():
    """Every Table 3 row: inside a window around it, n_m has least k = m + 1
    and is a record-setter with that depth."""
    knobs()
    for m, n in read_golden("table3_records.txt"):
        m, n = int(m), int(n)
        lo, hi = max(3, n - (1 << 16)), n + (1 << 16)
        g = esq.verify_range(lo, hi, per_n=True)
        assert int(g["per_n"][(n - g["n0"]) // 2]) == m + 1
        assert g["kmax_seen"] >= m + 1
        assert g["n_exceptions"] == 0


def test_calls_on_several_streams_share_scratch_blocks_safely():
    """Per-call scratch blocks are reused by later calls on the same stream
    and, after a device-side wait, by calls on other streams: many calls of
    three sizes (summary and per-n) enqueued over four streams without
    synchronising all equal the same calls made one at a time."""
    knobs()
    ivs = [((1 << 44) + 1, (1 << 44) + (1 << 24)), ((1 << 40) + 7, (1 << 40) + (1 << 20) + 3),
           (3, 1 << 21)]
    ref = [esq.verify_range(a, b, per_n=True) for a, b in ivs]
    streams = [torch.cuda.Stream() for _ in range(4)]
    pend = []
    for i in range(24):
        a, b = ivs[(i * 7) % 3]
        pend.append((ivs.index((a, b)), esq.verify_range_async(a, b, per_n=(i % 5 == 0),
                                                               stream=streams[i % 4])))
    for j, p in pend:
        r = p.result()
        assert r["hist"] == ref[j]["hist"] and r["records"] == ref[j]["records"]
        if "per_n" in r:
            assert torch.equal(r["per_n"], ref[j]["per_n"])


def test_errors_are_reported():
    with pytest.raises(esq.EsqError):
        esq.verify_range(3, 100, kmax=64)
    with pytest.raises(esq.EsqError):
        esq.verify_range(3, esq.ESQ_MAX_HI + 2)
    with pytest.raises(esq.EsqError):
        esq.verify_range(3, 100, exceptions_cap=esq.ESQ_EXCEPTIONS_CAP_MAX + 1)
    L = esq.lib()
    assert L.esq_verify_range(100, 3, 0, None, None, None, None, 0, None) == -1


def test_phase_clock_and_ceilings():
    """The measurement hooks change no result: the phase clock counts every
    phase of the segment loop, and the ceiling microbenchmarks return
    plausible rates."""
    knobs()
    lo, hi = (1 << 40) + 1, (1 << 40) + 1 + (1 << 24)
    ref = esq.verify_range(lo, hi, per_n=True)
    esq.set_param("phase_clock", 1)
    try:
        esq.phase_take()
        g = esq.verify_range(lo, hi, per_n=True)
        ph = esq.phase_take()
        esq.sieve_segment(lo, hi)
        ph2 = esq.phase_take()
    finally:
        esq.set_param("phase_clock", 0)
    assert g["hist"] == ref["hist"] and torch.equal(g["per_n"], ref["per_n"])
    assert all(v > 0 for v in ph.values()) and all(v > 0 for v in ph2.values())
    assert esq.phase_take() == {"init": 0, "mark": 0, "search_or_store": 0}
    c = esq.measure_ceilings()
    for k in ("lds_write_b64_Bps", "lds_read_b64_Bps", "lds_or_b32_Bps"):
        assert 1e12 < c[k] < 1e15, (k, c[k])
    for k in ("valu_int32_ops_per_s", "valu_alignbit_ops_per_s", "valu_bcnt_ops_per_s"):
        assert 1e12 < c[k] < 1e15, (k, c[k])
    assert 1e12 < c["l2_read_Bps"] < 1e15
    # streaming writes to a buffer 8x the last-level cache: HBM-bound
    assert 1e12 < c["hbm_write_Bps"] < 1e13


def test_near_the_largest_supported_n():
    """Windows just below ESQ_MAX_HI = 2^56 (prime table up to 2^28) and at
    2^53, where doubles no longer hold every odd n: verify and sieve against
    the oracle."""
    esq.init(0, esq.ESQ_MAX_HI)
    knobs()
    top = esq.ESQ_MAX_HI - 1
    for lo, hi in ((top - 2 * 700, top), ((1 << 53) + 1, (1 << 53) + 1 + 2 * 600)):
        g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=16)
        o = oracle.verify_range(lo, hi, per_n=True)
        assert_same(g, o)
        m0, n, w = esq.sieve_segment(lo, hi)
        om0, on, ow = oracle.sieve_bits(lo, hi)
        assert (m0, n) == (om0, on)
        assert np.array_equal(words_np(w), ow)


@pytest.mark.parametrize("kmax", [1, 3])
def test_kmax_at_most_kh_needs_no_tail_list(kmax):
    """With the search limit at or below the in-LDS depth, the n left after
    the LDS steps are exceptions already counted: a tail list far smaller
    than their number changes nothing in the counts, records (with their
    exception kind) or per-n bytes; a listed exception set that did not fit
    is reported as incomplete, never as wrong."""
    cap = 1 << 12 if kmax == 1 else 1 << 6
    knobs(tail_cap=cap)
    lo, hi = 3, (1 << 19) + 1
    o = oracle.verify_range(lo, hi, kmax=kmax, per_n=True, exc_cap=1 << 20)
    assert o["n_exceptions"] > 4 * cap
    g = esq.verify_range(lo, hi, kmax=kmax, per_n=True)
    assert g["status"] == 0
    assert_same(g, o)
    assert g["records"][-1][1] == 0 and g["record_flags"][-1] == esq.RECORD_KMAX_LIMIT
    s = esq.verify_range(lo, hi, kmax=kmax)
    assert s["hist"] == o["hist"] and s["records"] == o["records"] and s["status"] == 0
    e = esq.verify_range(lo, hi, kmax=kmax, exceptions_cap=64, check=False)
    assert e["status"] in (0, esq.STATUS_EXCEPTIONS_INCOMPLETE)
    assert e["hist"] == o["hist"] and e["records"] == o["records"]
    if e["status"] == 0:
        assert e["exceptions"] == o["exceptions"][:64]
    knobs()
    e = esq.verify_range(lo, hi, kmax=kmax, exceptions_cap=64)
    assert e["exceptions"] == o["exceptions"][:64]


@pytest.mark.parametrize("kh,seg_log2", [(13, 18), (8, 12), (4, 10), (13, 10)])
def test_region_origin_near_zero(kh, seg_log2):
    """The search's regions start one odd index below a word boundary: the
    region whose first word starts at odd index 0 (its bit 0 is odd index -1,
    not positive) and the regions below 0, against the oracle, per n, at
    several halo depths."""
    knobs(kh=kh, seg_log2=seg_log2)
    halo = (1 << (kh - 1)) if kh >= 7 else 64
    for lo, hi in ((2 * halo + 1, 2 * halo + 1 + 2 * 5000), (1, 2 * halo + 2 * 3000),
                   (2 * halo - 63, 2 * halo + 2 * 700)):
        g = esq.verify_range(lo, hi, per_n=True, exceptions_cap=64)
        o = oracle.verify_range(lo, hi, per_n=True)
        assert_same(g, o)
    knobs()
