// Host side of libesq: the C-ABI declared in include/esq.h.
//
// The library keeps, per process, one context on one device: the odd primes
// up to isqrt(max_hi) (Algorithm 1's prime list, Section 3 of the paper), the
// pattern table of odd multiples of 9, 25, 49 and 121, and cached lane-task
// tables for the medium primes.  Each call plans its segments on the host,
// allocates scratch in stream order on the caller's stream, enqueues the
// kernels and returns; nothing here waits for the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "esq.h"
#include "esq_internal.h"

using namespace esq;

namespace {

thread_local std::string t_err;

int fail(int code, const std::string& msg)
{
    t_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(ESQ_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Params {
    int seg_log2 = 18;
    int kh = 13;
    int block = 256;
    int entry_hits = 16;
    int64_t tail_cap = 1 << 20;
    int profile = 0;
};

struct MedTable {
    MedEntry* d = nullptr;
    uint32_t n = 0;
};

struct Ctx {
    int device = -1;
    uint64_t max_hi = 0;
    uint64_t plimit = 0;            // every odd prime <= plimit is in `primes`
    std::vector<uint32_t> primes;   // odd primes ascending (3, 5, 7, ...)
    std::vector<double> inv_pref;   // inv_pref[i] = sum over t < i of 1 / primes[t]^2
    uint32_t* d_primes = nullptr;
    uint64_t* d_wheel = nullptr;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, MedTable> med;
};

std::mutex g_mu;
Ctx* g_ctx = nullptr;
Params g_par;

// event pairs recorded around segment-kernel launches while "profile" is on
std::mutex g_prof_mu;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_open, g_prof_pool;

int prof_begin(hipStream_t s, std::pair<hipEvent_t, hipEvent_t>* ev)
{
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_pool.empty()) {
            *ev = g_prof_pool.back();
            g_prof_pool.pop_back();
        } else {
            ev->first = ev->second = nullptr;
        }
    }
    if (!ev->first) {
        if (hipEventCreate(&ev->first) != hipSuccess || hipEventCreate(&ev->second) != hipSuccess)
            return fail(ESQ_EHIP, "hipEventCreate");
    }
    if (hipEventRecord(ev->first, s) != hipSuccess)
        return fail(ESQ_EHIP, "hipEventRecord");
    return ESQ_OK;
}

void prof_end(hipStream_t s, const std::pair<hipEvent_t, hipEvent_t>& ev)
{
    (void)hipEventRecord(ev.second, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_open.push_back(ev);
}

uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = (uint64_t)std::sqrt((double)x);
    while (r * r > x)
        r--;
    while ((r + 1) * (r + 1) <= x)
        r++;
    return r;
}

// Odd primes up to `limit` (sieve of Eratosthenes over the odd numbers).
std::vector<uint32_t> odd_primes_upto(uint64_t limit)
{
    std::vector<uint32_t> out;
    if (limit < 3)
        return out;
    const uint64_t nodd = (limit - 1) / 2;  // odd numbers 3 .. limit: index i -> 2i + 3
    std::vector<uint8_t> comp(nodd, 0);
    for (uint64_t i = 0; i < nodd; i++) {
        if (comp[i])
            continue;
        const uint64_t p = 2 * i + 3;
        if (p * p > limit)
            break;
        for (uint64_t m = p * p; m <= limit; m += 2 * p)
            comp[(m - 3) / 2] = 1;
    }
    out.reserve((size_t)(limit / std::max(1.0, std::log((double)limit))) + 16);
    for (uint64_t i = 0; i < nodd; i++)
        if (!comp[i])
            out.push_back((uint32_t)(2 * i + 3));
    return out;
}

void free_ctx(Ctx* c)
{
    if (!c)
        return;
    if (c->device >= 0)
        (void)hipSetDevice(c->device);
    for (auto& kv : c->med)
        if (kv.second.d)
            (void)hipFree(kv.second.d);
    if (c->d_primes)
        (void)hipFree(c->d_primes);
    if (c->d_wheel)
        (void)hipFree(c->d_wheel);
    delete c;
}

// index of the first prime > x
uint32_t prime_upper(const Ctx* c, uint64_t x)
{
    if (x >= 0xffffffffull)
        return (uint32_t)c->primes.size();
    return (uint32_t)(std::upper_bound(c->primes.begin(), c->primes.end(), (uint32_t)x) -
                      c->primes.begin());
}

// Lane-tasks for the medium primes of a region of rw words: prime i (13 is
// i = 0) with up to h = ceil(R / q) marks per region is split into
// c = ceil(h / entry_hits) tasks; task v marks f + (v + c t) q, t >= 0.
int get_med_table(Ctx* c, uint32_t rw, uint32_t nmed, uint32_t entry_hits, MedTable** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple(rw, nmed, entry_hits);
    auto it = c->med.find(key);
    if (it != c->med.end()) {
        *out = &it->second;
        return ESQ_OK;
    }
    const uint64_t R = (uint64_t)rw * 64;
    std::vector<std::pair<uint64_t, MedEntry>> tasks;
    for (uint32_t i = 0; i < nmed; i++) {
        const uint64_t p = c->primes[4 + i];
        const uint64_t q = p * p;
        const uint64_t h = (R + q - 1) / q;
        uint64_t parts = std::max<uint64_t>(1, (h + entry_hits - 1) / entry_hits);
        parts = std::min<uint64_t>(parts, 65535);
        for (uint64_t v = 0; v < parts; v++) {
            MedEntry e;
            e.idx = i;
            e.vc = (uint32_t)v | ((uint32_t)parts << 16);
            tasks.push_back({(h + parts - 1) / parts, e});
        }
    }
    // lanes of one wave get tasks of similar length
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<MedEntry> host(tasks.size());
    for (size_t i = 0; i < tasks.size(); i++)
        host[i] = tasks[i].second;
    MedTable t;
    t.n = (uint32_t)host.size();
    if (t.n) {
        hipError_t e = hipMalloc(&t.d, host.size() * sizeof(MedEntry));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(medium table)");
        e = hipMemcpy(t.d, host.data(), host.size() * sizeof(MedEntry), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(t.d);
            return hip_fail(e, "hipMemcpy(medium table)");
        }
    }
    auto res = c->med.emplace(key, t);
    *out = &res.first->second;
    return ESQ_OK;
}

// Geometry of one call, shared by both entry points.
struct Plan {
    uint32_t S = 0, log2S = 0, hlo_words = 0, hup_words = 0, rw = 0, nseg = 0;
    int64_t A0 = 0;
    uint32_t med_end = 4, nmed = 0, b_begin = 0, b_end = 0, n_heavy = 0;
    uint64_t E = 0, capacity = 0;
};

int make_plan(const Ctx* c, const Params& par, int64_t A0, uint64_t span_words,
              uint32_t hlo_words, uint32_t hup_words, uint64_t pmax, Plan* pl)
{
    Plan p;
    p.log2S = (uint32_t)par.seg_log2;
    p.S = 1u << p.log2S;
    p.hlo_words = hlo_words;
    p.hup_words = hup_words;
    p.rw = hlo_words + p.S / 64 + hup_words;
    p.A0 = A0;
    const uint64_t nseg = (span_words + p.S / 64 - 1) / (p.S / 64);
    if (nseg > 0x7fffffffull)
        return fail(ESQ_ERANGE, "too many segments");
    p.nseg = (uint32_t)nseg;
    if (pmax > c->plimit)
        return fail(ESQ_ERANGE, "range exceeds the prime table built by esq_init");
    const uint64_t R = (uint64_t)p.rw * 64;
    const uint32_t pmax_end = prime_upper(c, pmax);
    uint32_t med_end = std::min(prime_upper(c, isqrt_u64(R)), pmax_end);
    med_end = std::max<uint32_t>(med_end, 4);
    p.med_end = med_end;
    p.nmed = std::min<uint32_t>(med_end - 4, (uint32_t)kMaxMedium);
    p.med_end = 4 + p.nmed;
    p.b_begin = p.med_end;
    p.b_end = std::max(pmax_end, p.b_begin);
    p.E = (uint64_t)(p.nseg - (p.nseg ? 1 : 0)) * p.S + R;
    if (p.b_end > p.b_begin) {
        const uint32_t heavy_end = prime_upper(c, isqrt_u64(p.E / 64));
        p.n_heavy = heavy_end > p.b_begin ? std::min(heavy_end, p.b_end) - p.b_begin : 0;
        const double sum_inv = c->inv_pref[p.b_end] - c->inv_pref[p.b_begin];
        const double hits = std::ceil((double)p.E * sum_inv * (1.0 + 1e-9)) + (double)(p.b_end - p.b_begin);
        // a hit lies in up to ceil(R / S) overlapping segment regions
        const double dup = std::ceil((double)R / (double)p.S);
        const double cap = dup * hits + 1024.0;
        if (cap >= 4294967295.0)
            return fail(ESQ_ERANGE, "range too long for one call (large-prime hit lists)");
        p.capacity = (uint64_t)cap;
    }
    *pl = p;
    return ESQ_OK;
}

uint32_t wheel_base(int64_t region_start)
{
    const int64_t g = region_start / 64;  // exact, region_start is a multiple of 64
    int64_t r = g % (int64_t)kWheelPeriod;
    if (r < 0)
        r += kWheelPeriod;
    return (uint32_t)r;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Scratch {
    char* base = nullptr;
    Acc* acc = nullptr;
    uint32_t *counts = nullptr, *cursor = nullptr, *offsets = nullptr, *entries = nullptr;
    unsigned long long* tail_n = nullptr;
    uint8_t* tail_d = nullptr;
};

int alloc_scratch(const Plan& p, uint64_t tail_cap, hipStream_t s, Scratch* sc)
{
    const bool buckets = p.b_end > p.b_begin;
    size_t off = 0;
    const size_t o_acc = off;
    off = align_up(off + sizeof(Acc));
    const size_t o_counts = off;
    off = align_up(off + (buckets ? (size_t)p.nseg * 4 : 0));
    const size_t o_cursor = off;
    off = align_up(off + (buckets ? (size_t)p.nseg * 4 : 0));
    const size_t o_offsets = off;
    off = align_up(off + (buckets ? (size_t)(p.nseg + 1) * 4 : 0));
    const size_t o_entries = off;
    off = align_up(off + (buckets ? (size_t)p.capacity * 4 : 0));
    const size_t o_tail_n = off;
    off = align_up(off + (size_t)tail_cap * 8);
    const size_t o_tail_d = off;
    off = align_up(off + (size_t)tail_cap);
    void* b = nullptr;
    hipError_t e = hipMallocAsync(&b, off, s);
    if (e != hipSuccess || !b)
        return fail(ESQ_ENOMEM, std::string("hipMallocAsync(scratch): ") + hipGetErrorString(e));
    sc->base = (char*)b;
    sc->acc = (Acc*)(sc->base + o_acc);
    if (buckets) {
        sc->counts = (uint32_t*)(sc->base + o_counts);
        sc->cursor = (uint32_t*)(sc->base + o_cursor);
        sc->offsets = (uint32_t*)(sc->base + o_offsets);
        sc->entries = (uint32_t*)(sc->base + o_entries);
    }
    sc->tail_n = (unsigned long long*)(sc->base + o_tail_n);
    sc->tail_d = (uint8_t*)(sc->base + o_tail_d);
    return ESQ_OK;
}

// Prepare + large-prime hit lists; shared by both entry points.
int enqueue_sieve_setup(const Ctx* c, const Plan& p, const Scratch& sc, hipStream_t s)
{
    const bool buckets = p.b_end > p.b_begin;
    hipError_t e = launch_prepare(sc.acc, buckets ? sc.counts : nullptr, sc.cursor, p.nseg, s);
    if (e != hipSuccess)
        return hip_fail(e, "k_prepare");
    if (!buckets || p.nseg == 0)
        return ESQ_OK;
    BucketParams bp;
    std::memset(&bp, 0, sizeof(bp));
    bp.primes = c->d_primes;
    bp.p_begin = p.b_begin;
    bp.n_heavy = p.n_heavy;
    bp.n_light = p.b_end - p.b_begin - p.n_heavy;
    bp.log2S = p.log2S;
    bp.overlap = p.rw * 64 - p.S;
    bp.nseg = p.nseg;
    bp.B0 = p.A0 - (int64_t)p.hlo_words * 64;
    bp.E = p.E;
    bp.counts = sc.counts;
    bp.cursor = sc.cursor;
    bp.offsets = sc.offsets;
    bp.entries = sc.entries;
    bp.capacity = p.capacity;
    bp.acc = sc.acc;
    if ((e = launch_bucket(bp, false, s)) != hipSuccess)
        return hip_fail(e, "k_bucket(count)");
    if ((e = launch_scan(sc.counts, sc.offsets, p.nseg, sc.acc, p.capacity, s)) != hipSuccess)
        return hip_fail(e, "k_scan");
    if ((e = launch_bucket(bp, true, s)) != hipSuccess)
        return hip_fail(e, "k_bucket(fill)");
    return ESQ_OK;
}

void fill_seg_params(const Ctx* c, const Plan& p, const Scratch& sc, const MedTable* mt,
                     SegParams* sp)
{
    std::memset(sp, 0, sizeof(*sp));
    sp->A0 = p.A0;
    sp->log2S = p.log2S;
    sp->hlo_words = p.hlo_words;
    sp->rw = p.rw;
    sp->nseg = p.nseg;
    sp->wheel_base0 = wheel_base(p.A0 - (int64_t)p.hlo_words * 64);
    sp->wheel_step = (uint32_t)((p.S / 64) % kWheelPeriod);
    sp->wheel = c->d_wheel;
    sp->primes = c->d_primes;
    sp->med_begin = 4;
    sp->nmed = p.nmed;
    sp->med = mt ? mt->d : nullptr;
    sp->n_med_entries = mt ? mt->n : 0;
    if (p.b_end > p.b_begin) {
        sp->bucket_off = sc.offsets;
        sp->bucket_ent = sc.entries;
        sp->bucket_cap = p.capacity;
    }
    sp->acc = sc.acc;
}

int snapshot(Ctx** c, Params* par)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ctx)
        return fail(ESQ_ENOINIT, "esq_init has not been called");
    *c = g_ctx;
    *par = g_par;
    hipError_t e = hipSetDevice(g_ctx->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    return ESQ_OK;
}

}  // namespace

extern "C" {

int esq_init(int device, uint64_t max_hi)
{
    t_err.clear();
    if (max_hi > ESQ_MAX_HI)
        return fail(ESQ_ERANGE, "max_hi above ESQ_MAX_HI");
    if (max_hi < 16)
        max_hi = 16;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ctx && g_ctx->device != device) {
        free_ctx(g_ctx);
        g_ctx = nullptr;
    }
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    bool fresh = false;
    if (!g_ctx) {
        g_ctx = new Ctx();
        g_ctx->device = device;
        fresh = true;
        if ((e = configure_kernels()) != hipSuccess) {
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return hip_fail(e, "hipFuncSetAttribute");
        }
        e = hipMalloc(&g_ctx->d_wheel, (size_t)(kWheelPeriod + kWheelExtra) * 8);
        if (e != hipSuccess) {
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return fail(ESQ_ENOMEM, "hipMalloc(wheel)");
        }
        if ((e = launch_wheel_build(g_ctx->d_wheel, nullptr)) != hipSuccess) {
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return hip_fail(e, "k_wheel_build");
        }
    }
    Ctx* c = g_ctx;
    const uint64_t need = isqrt_u64(max_hi) + 1;
    if (fresh || need > c->plimit) {
        std::vector<uint32_t> pr = odd_primes_upto(need);
        std::vector<double> pref(pr.size() + 1, 0.0);
        for (size_t i = 0; i < pr.size(); i++)
            pref[i + 1] = pref[i] + 1.0 / ((double)pr[i] * (double)pr[i]);
        uint32_t* d = nullptr;
        e = hipMalloc(&d, std::max<size_t>(pr.size(), 1) * 4);
        if (e != hipSuccess)
            return fail(ESQ_ENOMEM, "hipMalloc(primes)");
        if (!pr.empty() && (e = hipMemcpy(d, pr.data(), pr.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(e, "hipMemcpy(primes)");
        }
        if (c->d_primes) {
            (void)hipDeviceSynchronize();
            (void)hipFree(c->d_primes);
        }
        c->d_primes = d;
        c->primes.swap(pr);
        c->inv_pref.swap(pref);
        c->plimit = need;
    }
    c->max_hi = std::max(c->max_hi, max_hi);
    if ((e = hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(e, "hipDeviceSynchronize(init)");
    return ESQ_OK;
}

int esq_sieve_segment(uint64_t lo, uint64_t hi, uint64_t* d_bits, void* stream)
{
    t_err.clear();
    Ctx* c;
    Params par;
    int rc = snapshot(&c, &par);
    if (rc)
        return rc;
    if (lo > hi)
        return fail(ESQ_EINVAL, "lo > hi");
    if (hi > c->max_hi)
        return fail(ESQ_ERANGE, "hi above the max_hi given to esq_init");
    if (lo < 1)
        lo = 1;
    const uint64_t m0 = lo | 1;
    if (hi <= m0)
        return ESQ_OK;
    const uint64_t n_bits = (hi - m0 + 1) / 2;
    if (!d_bits)
        return fail(ESQ_EINVAL, "d_bits is null");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t I0 = (m0 - 1) / 2;
    const int64_t A0 = (int64_t)(I0 & ~63ull);
    const uint64_t n_out = (n_bits + 63) / 64;
    const uint64_t m_last = m0 + 2 * (n_bits - 1);
    Plan p;
    if ((rc = make_plan(c, par, A0, n_out, 0, 1, isqrt_u64(m_last), &p)))
        return rc;
    MedTable* mt = nullptr;
    if (p.nmed && (rc = get_med_table(c, p.rw, p.nmed, (uint32_t)par.entry_hits, &mt)))
        return rc;
    Scratch sc;
    if ((rc = alloc_scratch(p, 1, s, &sc)))
        return rc;
    if ((rc = enqueue_sieve_setup(c, p, sc, s))) {
        (void)hipFreeAsync(sc.base, s);
        return rc;
    }
    SegParams sp;
    fill_seg_params(c, p, sc, mt, &sp);
    sp.out_bits = d_bits;
    sp.n_bits = n_bits;
    sp.out_shift = (uint32_t)(I0 - (uint64_t)A0);
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (par.profile && (rc = prof_begin(s, &ev))) {
        (void)hipFreeAsync(sc.base, s);
        return rc;
    }
    hipError_t e = launch_segment(sp, 2, (uint32_t)par.block, s);
    if (par.profile)
        prof_end(s, ev);
    (void)hipFreeAsync(sc.base, s);
    if (e != hipSuccess)
        return hip_fail(e, "k_segment(sieve)");
    return ESQ_OK;
}

int esq_verify_range(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t* d_out_mink,
                     esq_summary* out_summary, esq_record* out_records, uint64_t* out_exceptions,
                     uint64_t exceptions_cap, void* stream)
{
    t_err.clear();
    Ctx* c;
    Params par;
    int rc = snapshot(&c, &par);
    if (rc)
        return rc;
    if (!out_summary)
        return fail(ESQ_EINVAL, "out_summary is null");
    if (kmax > 63)
        return fail(ESQ_EINVAL, "kmax > 63");
    if (lo > hi)
        return fail(ESQ_EINVAL, "lo > hi");
    if (exceptions_cap > ESQ_EXCEPTIONS_CAP_MAX)
        return fail(ESQ_EINVAL, "exceptions_cap above ESQ_EXCEPTIONS_CAP_MAX");
    if (exceptions_cap && !out_exceptions)
        return fail(ESQ_EINVAL, "out_exceptions is null but exceptions_cap > 0");
    if (hi > c->max_hi)
        return fail(ESQ_ERANGE, "hi above the max_hi given to esq_init");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t n0 = std::max<uint64_t>(lo, 3) | 1;
    const uint64_t n_odd = hi > n0 ? (hi - n0 + 1) / 2 : 0;
    const uint32_t kmax_eff = kmax ? kmax : 63;
    const uint32_t klds = std::min<uint32_t>(kmax_eff, (uint32_t)par.kh);
    const uint32_t hbits = klds >= 7 ? (1u << (klds - 1)) : 64u;
    const uint64_t I0 = (n0 - 1) / 2, I1 = I0 + n_odd;
    const int64_t A0 = (int64_t)(I0 & ~63ull);
    Plan p;
    if (n_odd) {
        const uint64_t span = (I1 - (uint64_t)A0 + 63) / 64;
        const uint64_t n_last = n0 + 2 * (n_odd - 1);
        if ((rc = make_plan(c, par, A0, span, hbits / 64, 0, isqrt_u64(n_last - 2), &p)))
            return rc;
    }
    MedTable* mt = nullptr;
    if (n_odd && p.nmed && (rc = get_med_table(c, p.rw, p.nmed, (uint32_t)par.entry_hits, &mt)))
        return rc;
    const uint64_t tail_cap = std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)par.tail_cap, n_odd));
    Scratch sc;
    if ((rc = alloc_scratch(p, tail_cap, s, &sc)))
        return rc;
    hipError_t e;
    if (n_odd) {
        if ((rc = enqueue_sieve_setup(c, p, sc, s))) {
            (void)hipFreeAsync(sc.base, s);
            return rc;
        }
        SegParams sp;
        fill_seg_params(c, p, sc, mt, &sp);
        sp.I0 = I0;
        sp.I1 = I1;
        sp.k_lds = klds;
        sp.tail_n = sc.tail_n;
        sp.tail_cap = tail_cap;
        sp.out_mink = d_out_mink;
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (par.profile && (rc = prof_begin(s, &ev))) {
            (void)hipFreeAsync(sc.base, s);
            return rc;
        }
        e = launch_segment(sp, d_out_mink ? 1 : 0, (uint32_t)par.block, s);
        if (par.profile)
            prof_end(s, ev);
        if (e != hipSuccess) {
            (void)hipFreeAsync(sc.base, s);
            return hip_fail(e, "k_segment");
        }
        TailParams tp;
        std::memset(&tp, 0, sizeof(tp));
        tp.acc = sc.acc;
        tp.tail_n = sc.tail_n;
        tp.tail_d = sc.tail_d;
        tp.tail_cap = tail_cap;
        tp.primes = c->d_primes;
        tp.nprimes = (uint32_t)c->primes.size();
        tp.k_lds = klds;
        tp.kmax_eff = kmax_eff;
        tp.I0 = I0;
        tp.out_mink = d_out_mink;
        if ((e = launch_tail(tp, s)) != hipSuccess) {
            (void)hipFreeAsync(sc.base, s);
            return hip_fail(e, "k_tail");
        }
    } else {
        if ((e = launch_prepare(sc.acc, nullptr, nullptr, 0, s)) != hipSuccess) {
            (void)hipFreeAsync(sc.base, s);
            return hip_fail(e, "k_prepare");
        }
    }
    FinParams fp;
    std::memset(&fp, 0, sizeof(fp));
    fp.acc = sc.acc;
    fp.tail_n = sc.tail_n;
    fp.tail_d = sc.tail_d;
    fp.tail_cap = tail_cap;
    fp.n_odd = n_odd;
    fp.I0 = I0;
    fp.k_lds = n_odd ? klds : 0;
    fp.out_summary = out_summary;
    fp.out_records = out_records;
    fp.out_exceptions = out_exceptions;
    fp.exc_cap = exceptions_cap;
    e = launch_finalize(fp, s);
    (void)hipFreeAsync(sc.base, s);
    if (e != hipSuccess)
        return hip_fail(e, "k_finalize");
    return ESQ_OK;
}

int esq_set_param(const char* name, int64_t value)
{
    t_err.clear();
    if (!name)
        return fail(ESQ_EINVAL, "null name");
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string n(name);
    if (n == "seg_log2") {
        if (value < kMinSegLog2 || value > kMaxSegLog2)
            return fail(ESQ_EINVAL, "seg_log2 out of range");
        g_par.seg_log2 = (int)value;
    } else if (n == "kh") {
        if (value < 1 || value > kMaxKh)
            return fail(ESQ_EINVAL, "kh out of range");
        g_par.kh = (int)value;
    } else if (n == "block") {
        if (value < 64 || value > 1024 || value % 64)
            return fail(ESQ_EINVAL, "block out of range");
        g_par.block = (int)value;
    } else if (n == "entry_hits") {
        if (value < 1 || value > 4096)
            return fail(ESQ_EINVAL, "entry_hits out of range");
        g_par.entry_hits = (int)value;
    } else if (n == "profile") {
        if (value < 0 || value > 1)
            return fail(ESQ_EINVAL, "profile must be 0 or 1");
        g_par.profile = (int)value;
    } else if (n == "tail_cap") {
        if (value < 1 || value > (int64_t)1 << 30)
            return fail(ESQ_EINVAL, "tail_cap out of range");
        g_par.tail_cap = value;
    } else {
        return fail(ESQ_EINVAL, "unknown parameter " + n);
    }
    return ESQ_OK;
}

int64_t esq_get_param(const char* name)
{
    if (!name)
        return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string n(name);
    if (n == "seg_log2") return g_par.seg_log2;
    if (n == "kh") return g_par.kh;
    if (n == "block") return g_par.block;
    if (n == "entry_hits") return g_par.entry_hits;
    if (n == "tail_cap") return g_par.tail_cap;
    if (n == "profile") return g_par.profile;
    return -1;
}

int esq_profile_take(double* total_ms, uint64_t* launches)
{
    t_err.clear();
    if (!total_ms || !launches)
        return fail(ESQ_EINVAL, "null pointer");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> open;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        open.swap(g_prof_open);
    }
    double sum = 0.0;
    int rc = ESQ_OK;
    for (auto& ev : open) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.second) != hipSuccess ||
            hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess)
            rc = fail(ESQ_EHIP, "hipEventElapsedTime");
        sum += ms;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pool.insert(g_prof_pool.end(), open.begin(), open.end());
    }
    *total_ms = sum;
    *launches = open.size();
    return rc;
}

const char* esq_last_error(void) { return t_err.c_str(); }

void esq_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ctx) {
        (void)hipSetDevice(g_ctx->device);
        (void)hipDeviceSynchronize();
    }
    free_ctx(g_ctx);
    g_ctx = nullptr;
}

}  // extern "C"
