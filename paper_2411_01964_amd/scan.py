"""Long scans: verify [lo, hi) as a sequence of chunks, merging the per-chunk
aggregates exactly and keeping a resumable checkpoint.

The paper's run covers all odd n below 2^50 as consecutive intervals
(Section 3: intervals of 2^30 integers; Section 4: the whole run).  The
aggregates merge associatively: counts and sums add, the maximum is a max,
the record-setters of the union are the strict prefix maxima of the
concatenated record lists (an n without representation counting as deeper
than any k), and exceptions concatenate.

Checkpoint: one JSON line per finished chunk, {"scan_lo", "kmax", "lo", "hi",
"summary", "crc"}, where crc is the CRC-32 of the line's canonical JSON
without it.  On resume, lines are read in order while they are intact,
contiguous and checksummed; the rest of [lo, hi) is cut into chunks again
from the end of the last intact line, so a resumed scan may use another chunk
size or a larger hi.  A checkpoint of another scan (a different start or
kmax, or one reaching past hi) is rejected.  A chunk whose verification
raises is retried.
"""
from __future__ import annotations

import json
import os
import zlib

DEEPER = 1 << 30  # depth of an n without representation in record merging


def empty(lo=None):
    return {"n0": 0, "n_odd": 0, "hist": [0] * 65, "ksum": 0, "kmax_seen": 0,
            "records": [], "n_exceptions": 0, "exceptions": [], "status": 0}


def merge(a, b, exceptions_cap=1 << 16):
    """Aggregate of two consecutive ranges (a before b)."""
    out = empty()
    out["n0"] = a["n0"] if a["n_odd"] else b["n0"]
    out["n_odd"] = a["n_odd"] + b["n_odd"]
    out["hist"] = [x + y for x, y in zip(a["hist"], b["hist"])]
    out["ksum"] = a["ksum"] + b["ksum"]
    out["kmax_seen"] = max(a["kmax_seen"], b["kmax_seen"])
    best, recs = 0, []
    for n, k in list(a["records"]) + list(b["records"]):
        d = k if k else DEEPER
        if d > best:
            recs.append((int(n), int(k)))
            best = d
    out["records"] = recs
    out["n_exceptions"] = a["n_exceptions"] + b["n_exceptions"]
    out["exceptions"] = (list(a.get("exceptions", [])) + list(b.get("exceptions", [])))[:exceptions_cap]
    out["status"] = a.get("status", 0) | b.get("status", 0)
    return out


_KEYS = ("n0", "n_odd", "hist", "ksum", "kmax_seen", "records", "n_exceptions")


def _pick(summary):
    out = {k: summary[k] for k in _KEYS}
    out["exceptions"] = list(summary.get("exceptions", []))
    out["status"] = int(summary.get("status", 0))
    return out


def _canon(summary):
    keep = _pick(summary)
    keep["records"] = [list(r) for r in keep["records"]]
    return json.dumps(keep, sort_keys=True, separators=(",", ":"))


def _line(scan_lo, kmax, a, b, s):
    body = {"scan_lo": scan_lo, "kmax": kmax, "lo": a, "hi": b, "summary": json.loads(_canon(s))}
    crc = zlib.crc32(json.dumps(body, sort_keys=True, separators=(",", ":")).encode())
    body["crc"] = crc
    return json.dumps(body) + "\n"


def _read_checkpoint(path, lo, hi, kmax):
    """The intact, contiguous prefix of a checkpoint of the scan of [lo, ...)
    with this kmax, as [(a, b, summary)]; raises ValueError for a checkpoint
    of another scan."""
    done = []
    if not path or not os.path.exists(path):
        return done
    expect = lo
    with open(path) as f:
        for line in f:
            try:
                rec = json.loads(line)
                crc = rec.pop("crc")
                if zlib.crc32(json.dumps(rec, sort_keys=True, separators=(",", ":")).encode()) != crc:
                    break
                s = rec["summary"]
                a, b = int(rec["lo"]), int(rec["hi"])
            except (ValueError, KeyError, TypeError, AttributeError):
                break
            if rec.get("scan_lo") != lo or rec.get("kmax") != kmax:
                raise ValueError("checkpoint %s belongs to another scan (start %r, kmax %r; this "
                                 "scan: start %d, kmax %d)" % (path, rec.get("scan_lo"), rec.get("kmax"),
                                                                lo, kmax))
            if a != expect or b <= a:
                break
            if b > hi:
                raise ValueError("checkpoint %s reaches %d, past the end %d of this scan" % (path, b, hi))
            s["records"] = [tuple(r) for r in s["records"]]
            done.append((a, b, s))
            expect = b
    return done


def odd_count(lo, hi):
    """Number of odd n >= 3 in [lo, hi)."""
    n0 = max(int(lo), 3) | 1
    return (int(hi) - n0 + 1) // 2 if int(hi) > n0 else 0


def _gpu_verify_async(kmax, exceptions_cap):
    from . import esq

    def start(lo, hi):
        return esq.verify_range_async(lo, hi, kmax=kmax, exceptions_cap=exceptions_cap)
    return start


def scan(lo, hi, chunk=1 << 40, checkpoint=None, kmax=0, exceptions_cap=1024,
         verify_async=None, retries=2, progress=None):
    """Verify every odd n in [lo, hi), chunk integers at a time.

    verify_async(lo, hi) must enqueue one chunk and return an object whose
    result() gives the chunk's summary dict; the default runs
    esq_verify_range on the GPU.  The next chunk is enqueued before the
    previous one's result is read, so the device never waits for the host.
    Returns the merged summary."""
    if verify_async is None:
        verify_async = _gpu_verify_async(kmax, exceptions_cap)
    lo, hi, kmax = int(lo), int(hi), int(kmax)
    done = _read_checkpoint(checkpoint, lo, hi, kmax)
    total = empty()
    for _, _, s in done:
        total = merge(total, s)
    # the rest of the range, cut from the end of the intact prefix
    todo = []
    a = done[-1][1] if done else lo
    while a < hi:
        b = min(hi, a + chunk)
        todo.append((a, b))
        a = b
    if checkpoint:
        # rewrite the intact prefix so that a damaged tail is dropped
        with open(checkpoint + ".tmp", "w") as f:
            for a, b, s in done:
                f.write(_line(lo, kmax, a, b, s))
        os.replace(checkpoint + ".tmp", checkpoint)
    out = open(checkpoint, "a") if checkpoint else None
    try:
        pending = None
        for i in range(len(todo) + 1):
            nxt = None
            if i < len(todo):
                nxt = (todo[i], verify_async(*todo[i]))
            if pending is not None:
                (a, b), p = pending
                s = None
                for attempt in range(retries + 1):
                    try:
                        s = p.result() if attempt == 0 else verify_async(a, b).result()
                        break
                    except Exception:
                        if attempt == retries:
                            raise
                s = _pick(s)
                total = merge(total, s)
                if out:
                    out.write(_line(lo, kmax, a, b, s))
                    out.flush()
                if progress:
                    progress(a, b, total)
            pending = nxt
    finally:
        if out:
            out.close()
    if total["n_odd"] != odd_count(lo, hi):
        raise RuntimeError("merged scan covers %d odd n, [%d, %d) has %d"
                           % (total["n_odd"], lo, hi, odd_count(lo, hi)))
    return total
