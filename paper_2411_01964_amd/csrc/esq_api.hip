// Host side of libesq: the C-ABI declared in include/esq.h.
//
// The library keeps, per process, one context on one device: the odd primes
// up to isqrt(max_hi) (Algorithm 1's prime list, Section 3 of the paper), the
// pattern table of odd multiples of 9, 25, 49 and 121, and cached tables for
// the medium primes.  Each call plans its intervals and segments on the host,
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

// Device scratch of esq_verify_range_noalloc: a static array that every
// device holds from the library's load until the process ends.  In host code
// the name is a host-side stand-in, never a device address: host code uses
// the address that hipGetSymbolAddress gives per device at esq_init
// (g_scratch_ptr), never the name itself.
static __device__ __align__(256) char scratch[ESQ_NOALLOC_SCRATCH_MAX];

namespace {

constexpr int kMaxDevices = 64;
char* g_scratch_ptr[kMaxDevices];  // under g_mu: device address of `scratch` per device

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
    int sieve_seg_log2 = 20;  // Algorithm 1 alone: one workgroup per CU, loader and storer waves
    int kh = 13;
    int block = 512;          // segment kernel, summary mode
    int per_n_block = 1024;   // per-n mode: more waves in flight behind the byte stores
    int sieve_block = 1024;   // Algorithm 1 alone: likewise behind the bitmap stores
    int entry_hits = 12;
    int64_t tail_cap = 1 << 20;
    int profile = 0;
    int phase_clock = 0;
    int64_t medium_max = 4095;  // largest prime marked per segment (others: hit slots)
    int64_t bucket_cap = 0;     // hit slots per segment; 0 = from the expected count
    int64_t items_per_wg = 4;   // batch: work items per resident workgroup
    int64_t runs_per_wg = 1;    // one interval: runs per resident workgroup
    int64_t stagger = 72;       // segment kernel: start delay per workgroup slot (x 64 clocks)
    int64_t priority = 1;       // segment kernel: wave priority from the share of the run left
    int64_t cof_weight = 60;    // large primes: cost of a cofactor thread, % of a first-hit thread
};

struct MedTable {
    uint2* tasks = nullptr;
    uint2* medq = nullptr;
    uint32_t n_tasks = 0;
};

// A device block of per-call scratch kept by the library.  A call takes the
// block its stream used last (else one no call holds whose last use has
// completed on the device, else a new one), makes its stream wait for the
// block's last use (an event: nothing to wait for on the same stream), and
// records that event after its kernels.  Stream-ordered pool allocation and
// release of the same sizes blocked the host for about as long as a call's
// kernels run, so that the host could not queue calls ahead of the device.
struct ScratchBlock {
    char* p = nullptr;
    size_t cap = 0;
    hipEvent_t last = nullptr;      // recorded after each call that used the block
    hipStream_t stream = nullptr;   // the stream of that call
    bool taken = false;             // held by a call being enqueued
};
constexpr size_t kScratchBlocks = 16;
constexpr size_t kScratchCacheBytes = (size_t)4 << 30;

struct Ctx {
    int device = -1;
    int n_cu = 256;
    uint64_t max_hi = 0;
    uint64_t plimit = 0;            // every odd prime <= plimit is in `primes`
    std::vector<uint32_t> primes;   // odd primes ascending (3, 5, 7, ...)
    std::vector<double> inv_pref;   // inv_pref[i] = sum over t < i of 1 / primes[t]^2
    uint32_t* d_primes = nullptr;   // the primes, their coarse index, Barrett reciprocals
    uint32_t pidx_n = 0;
    size_t qinv_at = 0;             // offset (uint32 units) of the reciprocals in d_primes
    uint32_t n_qinv = 0;            // primes[0 .. n_qinv) have one
    uint64_t* d_wheel = nullptr;
    unsigned long long* d_phase = nullptr;  // phase-clock counters, at the end of the d_wheel allocation
    uint64_t* d_wheel2 = nullptr;
    uint64_t* d_wheel_s = nullptr;  // the two tables one position lower (search regions)
    uint64_t* d_wheel2_s = nullptr;
    hipMemPool_t pool = nullptr;    // per-call scratch when no cached block serves (stream-ordered)
    std::vector<ScratchBlock> scratch;  // per-call scratch blocks kept for reuse (under scr_mu)
    size_t scratch_bytes = 0;
    std::mutex scr_mu;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, uint32_t>, MedTable> med;
    std::map<std::tuple<int, uint32_t, size_t>, int> occupancy;  // (mode, block, LDS bytes) -> workgroups per CU
    uint64_t generation = 0;        // changes whenever a device table that a prepared batch holds is replaced
};

std::mutex g_mu;
Ctx* g_ctx = nullptr;
Params g_par;
uint64_t g_generation = 0;  // under g_mu: last generation handed out

// event pairs recorded around verify-kernel launches while "profile" is on
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

// Pinned host staging buffers for descriptor uploads: a buffer is reused only
// once the event recorded after its last copy has completed.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool taken = false;
};
std::mutex g_stage_mu;
std::vector<Staging> g_stage;

int stage_upload(const std::vector<std::pair<const void*, size_t>>& parts,
                 const std::vector<char*>& dsts, hipStream_t s)
{
    size_t total = 0;
    for (auto& p : parts)
        total += (p.second + 255) & ~(size_t)255;
    if (total == 0)
        return ESQ_OK;
    int idx = -1;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        for (size_t i = 0; i < g_stage.size(); i++) {
            Staging& st = g_stage[i];
            if (!st.taken && st.cap >= total && hipEventQuery(st.done) == hipSuccess) {
                st.taken = true;
                idx = (int)i;
                break;
            }
        }
        if (idx < 0) {
            Staging st;
            st.cap = std::max<size_t>(total, 1 << 16);
            if (hipHostMalloc(&st.host, st.cap, hipHostMallocDefault) != hipSuccess)
                return fail(ESQ_ENOMEM, "hipHostMalloc(staging)");
            if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
                (void)hipHostFree(st.host);
                return fail(ESQ_EHIP, "hipEventCreate(staging)");
            }
            st.taken = true;
            g_stage.push_back(st);
            idx = (int)g_stage.size() - 1;
        }
    }
    Staging st;
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        st = g_stage[idx];
    }
    size_t off = 0;
    int rc = ESQ_OK;
    for (size_t i = 0; i < parts.size(); i++) {
        std::memcpy((char*)st.host + off, parts[i].first, parts[i].second);
        hipError_t e = hipMemcpyAsync(dsts[i], (char*)st.host + off, parts[i].second,
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "hipMemcpyAsync(descriptors)");
            break;
        }
        off += (parts[i].second + 255) & ~(size_t)255;
    }
    (void)hipEventRecord(st.done, s);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage[idx].taken = false;
    return rc;
}

uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = (uint64_t)std::sqrt((double)x);
    while (r > 0 && r * r > x)
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
    for (auto& kv : c->med) {
        if (kv.second.tasks)
            (void)hipFree(kv.second.tasks);
        if (kv.second.medq)
            (void)hipFree(kv.second.medq);
    }
    if (c->d_primes)
        (void)hipFree(c->d_primes);
    if (c->d_wheel)
        (void)hipFree(c->d_wheel);  // d_wheel2 lives in the same allocation
    if (c->pool || !c->scratch.empty())
        (void)hipDeviceSynchronize();  // no call may still hold scratch
    for (ScratchBlock& b : c->scratch) {
        (void)hipFree(b.p);
        (void)hipEventDestroy(b.last);
    }
    if (c->pool)
        (void)hipMemPoolDestroy(c->pool);
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

// Medium primes primes[kFirstMedium .. med_end) for a region of rw words and segment
// length S: per prime (q, S mod q), and lane-tasks -- prime i with up to
// h = ceil(R / q) marks per region is split into c = ceil(h / entry_hits)
// tasks; task v marks f + v q + t c q, t >= 0.  A task is packed as
// x = v q | i << 21 (v q < R < 2^21; i < 2^11) and y = c q.
//
// Task e of the table is taken by thread e mod block.
int get_med_table_locked(Ctx* c, uint32_t rw, uint32_t log2S, uint32_t med_end, uint32_t entry_hits,
                         uint32_t block, MedTable** out)
{
    const auto key = std::make_tuple(rw, log2S, med_end, entry_hits, block);
    auto it = c->med.find(key);
    if (it != c->med.end()) {
        *out = &it->second;
        return ESQ_OK;
    }
    const uint64_t R = (uint64_t)rw * 64;
    const uint64_t S = 1ull << log2S;
    const uint32_t nmed = med_end - kFirstMedium;
    if (R >= (1u << 21) || nmed > (1u << 11))
        return fail(ESQ_EINVAL, "medium-prime task packing: region or prime count too large");
    std::vector<std::pair<uint64_t, uint2>> tasks;
    std::vector<uint2> medq(std::max<uint32_t>(nmed, 1));
    for (uint32_t i = 0; i < nmed; i++) {
        const uint64_t p = c->primes[kFirstMedium + i];
        const uint64_t q = p * p;
        medq[i].x = (uint32_t)q;
        medq[i].y = (uint32_t)(S % q);
        const uint64_t h = (R + q - 1) / q;
        const uint64_t parts = std::max<uint64_t>(1, (h + entry_hits - 1) / entry_hits);
        for (uint64_t v = 0; v < parts; v++) {
            // v q <= (h - 1) q < R; c q <= R + q when c > 1, else q
            uint2 t;
            t.x = (uint32_t)(v * q) | (i << 21);
            t.y = (uint32_t)(parts * q);
            tasks.push_back({(h + parts - 1) / parts, t});
        }
    }
    // lanes of one wave get tasks of similar length (dealing groups of 64 to
    // the waves by load, which evens out the waves' marking, measured 4%
    // slower: the waves that finish early hand their SIMD to other
    // workgroups' search)
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    std::vector<uint2> host(tasks.size());
    for (size_t i = 0; i < tasks.size(); i++)
        host[i] = tasks[i].second;
    MedTable t;
    t.n_tasks = (uint32_t)host.size();
    hipError_t e = hipMalloc(&t.medq, medq.size() * sizeof(uint2));
    if (e != hipSuccess)
        return hip_fail(e, "hipMalloc(medium primes)");
    if ((e = hipMemcpy(t.medq, medq.data(), medq.size() * sizeof(uint2), hipMemcpyHostToDevice)) !=
        hipSuccess) {
        (void)hipFree(t.medq);
        return hip_fail(e, "hipMemcpy(medium primes)");
    }
    if (t.n_tasks) {
        if ((e = hipMalloc(&t.tasks, host.size() * sizeof(uint2))) != hipSuccess) {
            (void)hipFree(t.medq);
            return hip_fail(e, "hipMalloc(medium tasks)");
        }
        if ((e = hipMemcpy(t.tasks, host.data(), host.size() * sizeof(uint2),
                           hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(t.medq);
            (void)hipFree(t.tasks);
            return hip_fail(e, "hipMemcpy(medium tasks)");
        }
    }
    auto res = c->med.emplace(key, t);
    *out = &res.first->second;
    return ESQ_OK;
}

int get_med_table(Ctx* c, uint32_t rw, uint32_t log2S, uint32_t med_end, uint32_t entry_hits,
                  uint32_t block, MedTable** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return get_med_table_locked(c, rw, log2S, med_end, entry_hits, block, out);
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

// End of the medium primes for the knobs: primes[kFirstMedium .. end) are the
// odd primes 17 .. medium_max present in the table.
uint32_t medium_end(const Ctx* c, const Params& par)
{
    uint32_t e = std::max<uint32_t>(kFirstMedium, prime_upper(c, (uint64_t)par.medium_max));
    return std::min<uint32_t>(e, kFirstMedium + (uint32_t)kMaxMedium);
}

// Threads per workgroup of the segment kernel in a mode (0 summary, 1 per-n,
// 2 sieve alone) for a launch of n_iv intervals: per-n batches of many (short)
// intervals keep the summary block size, which keeps more workgroups resident.
uint32_t block_for(const Params& par, int mode, uint32_t n_iv)
{
    return (uint32_t)(mode == 2 ? par.sieve_block : mode == 1 && n_iv == 1 ? par.per_n_block : par.block);
}

// The medium-prime tables of the verify geometry for the current knobs (at
// the summary and the per-n block size), made at set-up (esq_init,
// esq_set_param; g_mu held) so that calls find them resident.
int prebuild_med_table(Ctx* c, const Params& par)
{
    const uint32_t med_end = medium_end(c, par);
    if (med_end <= kFirstMedium)
        return ESQ_OK;
    const uint32_t hlo = (par.kh >= 7 ? (1u << (par.kh - 1)) : 64u) / 64;
    const uint32_t rw = hlo + (uint32_t)((1ull << par.seg_log2) / 64);
    MedTable* mt = nullptr;
    for (int mode = 0; mode < 2; mode++) {
        const int rc = get_med_table_locked(c, rw, (uint32_t)par.seg_log2, med_end, (uint32_t)par.entry_hits,
                                            block_for(par, mode, 1), &mt);
        if (rc)
            return rc;
    }
    return ESQ_OK;
}

// One interval to process, in odd-index terms: verify -> the n-indices
// [I0, I1); sieve -> the m-indices of the output bits.
struct Req {
    uint64_t I0, I1;
    uint8_t* out_mink;
    uint64_t* out_bits;
};

// A launch planned on the host: geometry, descriptors, scratch layout.
struct Planned {
    Launch L;
    int mode = 0;
    std::vector<Interval> ivs;
    std::vector<uint4> items;
    uint32_t n_heavy = 0, max_direct = 0, max_cof = 0, grid = 0, block = 256;
    bool any_bucket = false;
    uint64_t nseg_total = 0;
    size_t bytes = 0, o_iv = 0, o_acc = 0, o_items = 0, o_bcnt = 0, o_bslot = 0, o_misc = 0;
    size_t o_tn = 0, o_tiv = 0, o_td = 0;
};

// Plan one launch over `reqs` (mode 0/1 verify, 2 sieve).
int plan(Ctx* c, const Params& par, int mode, uint32_t kmax, const std::vector<Req>& reqs,
         bool exc_list, Planned* P, bool no_alloc = false)
{
    const uint32_t n_iv = (uint32_t)reqs.size();
    const uint32_t log2S = (uint32_t)(mode == 2 ? par.sieve_seg_log2 : par.seg_log2);
    const uint32_t blk = block_for(par, mode, n_iv);
    const uint64_t S = 1ull << log2S;
    const uint32_t SW = (uint32_t)(S / 64);
    const uint32_t kmax_eff = kmax ? kmax : 63;
    const uint32_t klds = std::min<uint32_t>(kmax_eff, (uint32_t)par.kh);
    // The halo below a segment holds the candidates of depth up to kh, also
    // when kmax is smaller (a larger halo is harmless): the geometry, and with
    // it the medium-prime tables, depends on the knobs only.
    uint32_t hlo = 0, hup = 0;
    if (mode == 2) {
        hup = 1;
    } else {
        hlo = (par.kh >= 7 ? (1u << (par.kh - 1)) : 64u) / 64;
    }
    const uint32_t rw = hlo + SW + hup;
    const uint64_t R = (uint64_t)rw * 64;

    // per-interval geometry
    std::vector<Interval>& ivs = P->ivs;
    ivs.assign(n_iv, Interval());
    uint64_t nseg_total = 0, pmax_all = 0;
    std::vector<uint64_t> pmax(n_iv, 0);
    for (uint32_t i = 0; i < n_iv; i++) {
        const Req& r = reqs[i];
        Interval& v = ivs[i];
        std::memset(&v, 0, sizeof(v));
        v.I0 = r.I0;
        v.I1 = r.I1;
        v.A0 = (int64_t)(r.I0 & ~63ull);
        v.out_mink = r.out_mink;
        v.out_bits = r.out_bits;
        v.out_shift = (uint32_t)(r.I0 - (uint64_t)v.A0);
        if (r.I1 <= r.I0)
            continue;
        uint64_t nseg;
        if (mode == 2) {
            const uint64_t n_out = (r.I1 - r.I0 + 63) / 64;
            nseg = (n_out + SW - 1) / SW;
            pmax[i] = isqrt_u64(2 * (r.I1 - 1) + 1);                // last odd m
        } else {
            nseg = (r.I1 - (uint64_t)v.A0 + S - 1) / S;
            const uint64_t n_last = 2 * (r.I1 - 1) + 1;
            pmax[i] = n_last >= 3 ? isqrt_u64(n_last - 2) : 0;       // largest candidate
        }
        if (pmax[i] > c->plimit)
            return fail(ESQ_ERANGE, "range exceeds the prime table built by esq_init");
        v.nseg = (uint32_t)nseg;
        v.seg_base = (uint32_t)nseg_total;
        nseg_total += nseg;
        if (nseg_total > 0x7fffffffull)
            return fail(ESQ_ERANGE, "too many segments in one call");
        v.wheel_base0 = wheel_base(v.A0 - (int64_t)hlo * 64);
        pmax_all = std::max(pmax_all, pmax[i]);
    }

    // medium primes: 17 .. medium_max, whatever the interval (a prime whose
    // square exceeds every candidate marks only numbers no n looks at, or
    // none), so that the tables depend on the knobs only
    const uint32_t med_end = medium_end(c, par);
    // Bucket primes up to P0 take one first-hit computation (a 64-bit
    // modulo) each; the primes above P0 are found from their cofactors, one
    // thread per odd j <= m_hi / P0^2 (two square roots, mostly an empty range
    // for a short interval).  When the launch's direct threads at P0 = 2^20
    // fit in one pass of the device, the pass is latency-bound and 2^20 is
    // kept; otherwise (many intervals) P0, a power of 2^(1/2) in [2^10, 2^20],
    // minimizes the work #direct + 0.6 #cofactors for the largest candidate.
    uint64_t m_hi_max = 0;
    uint32_t n_live = 0;
    for (uint32_t i = 0; i < n_iv; i++) {
        const Interval& v = ivs[i];
        if (!v.nseg)
            continue;
        n_live++;
        const int64_t B0 = v.A0 - (int64_t)hlo * 64 - (mode == 2 ? 0 : 1);  // region bit 0
        const uint64_t E = (uint64_t)(v.nseg - 1) * S + R;
        m_hi_max = std::max(m_hi_max, 2 * (uint64_t)(B0 + (int64_t)E - 1) + 1);
    }
    uint64_t P0 = kCofactorPrime;
    const uint64_t direct_threads_full =
        (uint64_t)n_live * (uint64_t)(std::max(med_end, prime_upper(c, kCofactorPrime)) - med_end);
    if (direct_threads_full > (uint64_t)c->n_cu * 2048) {
        double best = 0;
        for (int h = 20; h <= 40; h++) {
            const uint64_t cand = (uint64_t)std::ldexp(1.0, h / 2) * (h % 2 ? 1.41421356 : 1.0);
            const uint32_t de = std::max(med_end, prime_upper(c, cand));
            const double n_direct = (double)(de - med_end);
            const double n_cofac = (double)m_hi_max / ((double)cand * (double)cand) / 2;
            const double cost = n_direct + 0.01 * (double)par.cof_weight * n_cofac;
            if (h == 20 || cost < best) {
                best = cost;
                P0 = cand;
            }
        }
    }
    const uint32_t direct_end = prime_upper(c, P0);
    uint32_t max_direct = 0, max_cof = 0;
    bool any_bucket = false;
    uint32_t pmax_end_all = med_end;
    uint64_t E_max = 0;
    for (uint32_t i = 0; i < n_iv; i++) {
        Interval& v = ivs[i];
        if (!v.nseg)
            continue;
        v.pmax_end = std::max(prime_upper(c, pmax[i]), med_end);
        pmax_end_all = std::max(pmax_end_all, v.pmax_end);
        v.b_direct_end = std::max(med_end, std::min(v.pmax_end, direct_end));
        if (v.pmax_end > v.b_direct_end) {
            const int64_t B0 = v.A0 - (int64_t)hlo * 64 - (mode == 2 ? 0 : 1);  // region bit 0
            const uint64_t E = (uint64_t)(v.nseg - 1) * S + R;
            const uint64_t m_hi = 2 * (uint64_t)(B0 + (int64_t)E - 1) + 1;
            const uint64_t pc = c->primes[v.b_direct_end];  // least cofactor-path prime
            const uint64_t jmax = m_hi / (pc * pc);
            v.n_cof = (uint32_t)((jmax + 1) / 2);
            // cofactor j's range holds about L / (2 sqrt(m j) ln p) primes:
            // the j with more than 4 share them over 8 lanes
            const double m_lo = std::max(1.0, 2.0 * (double)B0 + 1);
            const double span = 2.0 * (double)E;
            const double per_j = span / (2.0 * std::sqrt(m_lo) * std::log((double)pc));
            const double j_wide = (per_j / 4.0) * (per_j / 4.0);
            v.n_cof_wide = (uint32_t)std::min<double>(v.n_cof, std::floor((j_wide + 1) / 2));
        }
        if (v.pmax_end > med_end)
            any_bucket = true;
        max_direct = std::max(max_direct, v.b_direct_end - med_end);
        max_cof = std::max(max_cof, v.n_cof + 7 * v.n_cof_wide);  // cofactor threads
        E_max = std::max(E_max, (uint64_t)(v.nseg - 1) * S + R);
    }
    // bucket primes with more than 8 hits in the longest interval get a
    // group of lanes each
    uint32_t n_heavy = 0;
    if (any_bucket) {
        const uint32_t heavy_end = prime_upper(c, isqrt_u64(E_max / 8));
        n_heavy = heavy_end > med_end ? std::min(heavy_end - med_end, max_direct) : 0;
        max_direct -= n_heavy;
    }

    MedTable* mt = nullptr;
    int rc;
    if (med_end > kFirstMedium) {
        if (no_alloc) {
            // only a table made at set-up: making one here would allocate
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = c->med.find(std::make_tuple(rw, log2S, med_end, (uint32_t)par.entry_hits,
                                                  blk));
            if (it == c->med.end())
                return fail(ESQ_ENOMEM, "medium-prime tables for these knobs are not resident");
            mt = &it->second;
        } else if ((rc = get_med_table(c, rw, log2S, med_end, (uint32_t)par.entry_hits,
                                       blk, &mt))) {
            return rc;
        }
    }

    uint32_t cap = 0;
    if (any_bucket) {
        if (par.bucket_cap > 0) {
            cap = (uint32_t)par.bucket_cap;
        } else {
            const double expect = (double)R * (c->inv_pref[pmax_end_all] - c->inv_pref[med_end]);
            cap = (uint32_t)std::ceil(8.0 * expect + 32.0);
            cap = (cap + 7) & ~7u;
        }
    }

    // LDS of the segment kernel: bitmap + medium-prime tables (+ tasks if they fit)
    const uint32_t nmed = med_end - kFirstMedium;
    const uint32_t n_tasks = mt ? mt->n_tasks : 0;
    if (verify_lds_size(rw, nmed, 0, false, blk) > kVerifyLdsMax)
        return fail(ESQ_EINVAL, "segment too large for LDS with these medium primes");
    // per-n output is staged through LDS (1 KB contiguous per store) when the
    // staging area fits beside the bitmap
    const bool stage = mode == 1 && verify_lds_size(rw, nmed, 0, true, blk) <= kVerifyLdsMax;
    const size_t lds_base = verify_lds_size(rw, nmed, 0, stage, blk);
    auto occupancy = [&](size_t bytes) {
        std::lock_guard<std::mutex> lk(g_mu);
        const auto key = std::make_tuple(mode, blk, bytes);
        auto it = c->occupancy.find(key);
        if (it == c->occupancy.end())
            it = c->occupancy.emplace(key, verify_occupancy(mode, blk, bytes)).first;
        return it->second;
    };
    // the task table goes into LDS when it fits and costs no resident workgroup
    const size_t lds_with = verify_lds_size(rw, nmed, n_tasks, stage, blk);
    const bool tasks_in_lds = n_tasks == 0 || (lds_with <= kVerifyLdsMax &&
                                               occupancy(lds_with) >= occupancy(lds_base));
    const size_t lds_bytes = tasks_in_lds ? lds_with : lds_base;

    // work items: runs of consecutive segments
    const int occ = occupancy(lds_bytes);
    const uint64_t resident = (uint64_t)c->n_cu * (uint64_t)occ;
    std::vector<uint4>& items = P->items;
    items.clear();
    uint32_t n_items = 0;
    if (n_iv == 1) {
        // runs_per_wg runs per resident workgroup (a device-scope queue
        // operation costs microseconds, so runs stay few), each at most
        // kFlushSegs segments
        n_items = (uint32_t)std::min<uint64_t>(
            nseg_total, std::max<uint64_t>(resident * (uint64_t)par.runs_per_wg,
                                           (nseg_total + kFlushSegs - 1) / kFlushSegs));
    } else {
        const uint64_t target = std::max<uint64_t>(1, resident * (uint64_t)par.items_per_wg);
        const uint64_t run = std::min<uint64_t>(
            kFlushSegs, std::max<uint64_t>(1, (nseg_total + target - 1) / target));
        for (uint32_t i = 0; i < n_iv; i++)
            for (uint64_t b = 0; b < ivs[i].nseg; b += run) {
                uint4 x;
                x.x = i;
                x.y = (uint32_t)b;
                x.z = (uint32_t)std::min<uint64_t>(run, ivs[i].nseg - b);
                x.w = 0;
                items.push_back(x);
            }
        n_items = (uint32_t)items.size();
    }
    // no tail pass when the search limit is the in-LDS depth: the list then
    // only holds exceptions, and only when the call lists them
    const bool no_tail = klds >= kmax_eff;
    const uint64_t tail_cap = (mode == 2 || (no_tail && !exc_list))
                                  ? 1 : std::max<uint64_t>(1, (uint64_t)par.tail_cap);

    // scratch layout, one allocation
    size_t off = 0;
    P->o_iv = off;
    off = align_up(off + sizeof(Interval) * std::max<uint32_t>(n_iv, 1));
    P->o_acc = off;
    off = align_up(off + sizeof(Acc) * std::max<uint32_t>(n_iv, 1));
    P->o_items = off;
    off = align_up(off + sizeof(uint4) * items.size());
    P->o_bcnt = off;
    off = align_up(off + (any_bucket ? nseg_total * 4 : 0));
    P->o_bslot = off;
    off = align_up(off + (any_bucket ? nseg_total * cap * 4 : 0));
    P->o_misc = off;
    off = align_up(off + 64);
    P->o_tn = off;
    off = align_up(off + tail_cap * 8);
    P->o_tiv = off;
    off = align_up(off + tail_cap * 4);
    P->o_td = off;
    off = align_up(off + tail_cap);
    P->bytes = off;

    Launch& L = P->L;
    std::memset(&L, 0, sizeof(L));
    L.log2S = log2S;
    L.hlo_words = hlo;
    L.hup_words = hup;
    L.rw = rw;
    L.n_iv = n_iv;
    L.n_items = n_items;
    L.mode = (uint32_t)mode;
    L.med_end = med_end;
    L.n_tasks = n_tasks;
    L.tasks_in_lds = tasks_in_lds ? 1u : 0u;
    // the stagger pays in summary mode only (measured: the per-n and sieve
    // forms, bound by their HBM stores, are no faster with it)
    L.stagger = mode == 0 ? (uint32_t)par.stagger : 0u;
    L.priority = (uint32_t)par.priority;
    L.phase = par.phase_clock ? c->d_phase : nullptr;
    L.stage = stage ? 1u : 0u;
    L.k_lds = mode == 2 ? 0 : klds;
    L.kmax_eff = kmax_eff;
    L.exc_list = exc_list ? 1u : 0u;
    L.bucket_cap = cap;
    L.nprimes = (uint32_t)c->primes.size();
    L.primes = c->d_primes;
    L.pidx = c->d_primes + c->primes.size();
    L.pidx_n = c->pidx_n;
    L.qinv = reinterpret_cast<const uint64_t*>(c->d_primes + c->qinv_at);
    L.n_qinv = c->n_qinv;
    L.medq = mt ? mt->medq : nullptr;
    L.tasks = mt ? mt->tasks : nullptr;
    // search modes: a region's bit 0 is the odd index one below its word
    // boundary, so that a word of n-bits lines up with the bits of their
    // first candidates n - 2 (the search's first window needs no shift)
    L.origin = mode == 2 ? 0u : 1u;
    L.wheel = mode == 2 ? c->d_wheel : c->d_wheel_s;
    L.wheel2 = mode == 2 ? c->d_wheel2 : c->d_wheel2_s;
    L.tail_cap = tail_cap;
    P->mode = mode;
    P->n_heavy = n_heavy;
    P->max_direct = max_direct;
    P->max_cof = max_cof;
    P->any_bucket = any_bucket;
    P->nseg_total = nseg_total;
    P->grid = (uint32_t)std::min<uint64_t>(n_items, resident);
    P->block = blk;
    return ESQ_OK;
}

// Point the launch at its scratch (device pointer `base`).
void bind(Planned* P, char* base)
{
    Launch& L = P->L;
    Acc* accs = (Acc*)(base + P->o_acc);
    for (size_t i = 0; i < P->ivs.size(); i++)
        P->ivs[i].acc = accs + i;
    L.iv = (const Interval*)(base + P->o_iv);
    L.items = P->items.empty() ? nullptr : (const uint4*)(base + P->o_items);
    L.bucket_cnt = P->any_bucket ? (uint32_t*)(base + P->o_bcnt) : nullptr;
    L.bucket_slot = P->any_bucket ? (uint32_t*)(base + P->o_bslot) : nullptr;
    L.queue = (unsigned int*)(base + P->o_misc);
    L.tail_count = (unsigned long long*)(base + P->o_misc + 8);
    L.tail_n = (unsigned long long*)(base + P->o_tn);
    L.tail_iv = (uint32_t*)(base + P->o_tiv);
    L.tail_d = (uint8_t*)(base + P->o_td);
}

// The kernels of one launch, in stream order (no allocation, no copy): this
// is what a hipGraph captures.  With iv_by_value the single interval's
// descriptor travels as a kernel argument instead of being uploaded.
int launch_seq(const Planned& P, bool iv_by_value, bool profile, void* out_summaries,
               void* out_records, uint64_t* out_exceptions, uint64_t exc_cap, hipStream_t s)
{
    const Launch& L = P.L;
    Acc* accs = P.ivs.empty() ? nullptr : P.ivs[0].acc;
    hipError_t e;
    int rc;
    if ((e = launch_prepare(L, accs, iv_by_value ? &P.ivs[0] : nullptr, (uint32_t)P.nseg_total,
                            s)) != hipSuccess)
        return hip_fail(e, "k_prepare");
    if (P.any_bucket && (e = launch_bucket(L, P.n_heavy, P.max_direct, P.max_cof, s)) != hipSuccess)
        return hip_fail(e, "k_bucket");
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (profile && (rc = prof_begin(s, &ev)))
        return rc;
    e = launch_verify(L, P.grid, P.block, s);
    if (profile)
        prof_end(s, ev);
    if (e != hipSuccess)
        return hip_fail(e, "k_verify");
    if (P.mode != 2) {
        if ((e = launch_tail(L, s)) != hipSuccess)
            return hip_fail(e, "k_tail");
        if ((e = launch_finalize(L, out_summaries, out_records, out_exceptions, exc_cap, s)) !=
            hipSuccess)
            return hip_fail(e, "k_finalize");
    }
    return ESQ_OK;
}

// A cached scratch block of at least `bytes` for a call on stream s (see
// ScratchBlock), with s made to wait for the block's last use; -1 when none
// can be had (every block held or too small and the cache full, an
// allocation failure, or s capturing a graph): the caller then allocates from
// the pool.
int scratch_take(Ctx* c, size_t bytes, hipStream_t s, char** ptr)
{
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap_status) != hipSuccess || cap_status != hipStreamCaptureStatusNone)
        return -1;
    int idx = -1;
    hipEvent_t wait = nullptr;
    {
        std::lock_guard<std::mutex> lk(c->scr_mu);
        std::vector<ScratchBlock>& v = c->scratch;
        for (size_t i = 0; i < v.size() && idx < 0; i++)
            if (!v[i].taken && v[i].stream == s && v[i].cap >= bytes)
                idx = (int)i;
        for (size_t i = 0; i < v.size() && idx < 0; i++)
            if (!v[i].taken && v[i].cap >= bytes && hipEventQuery(v[i].last) == hipSuccess)
                idx = (int)i;
        if (idx < 0) {
            if (v.size() >= kScratchBlocks || c->scratch_bytes + bytes > kScratchCacheBytes)
                return -1;
            ScratchBlock b;
            b.cap = (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
            if (hipMalloc((void**)&b.p, b.cap) != hipSuccess) {
                (void)hipGetLastError();
                return -1;
            }
            if (hipEventCreateWithFlags(&b.last, hipEventDisableTiming) != hipSuccess) {
                (void)hipFree(b.p);
                return -1;
            }
            c->scratch_bytes += b.cap;
            v.push_back(b);
            idx = (int)v.size() - 1;
        }
        v[idx].taken = true;
        *ptr = v[idx].p;
        // the per-thread stream handle names another stream on each thread
        if (v[idx].stream != s || s == hipStreamPerThread)
            wait = v[idx].last;
    }
    // the block's last use, on another stream, completes before this call's
    // kernels (a block never used has an unrecorded event: no wait)
    if (wait && hipStreamWaitEvent(s, wait, 0) != hipSuccess) {
        std::lock_guard<std::mutex> lk(c->scr_mu);
        c->scratch[idx].taken = false;
        return -1;
    }
    return idx;
}

// Hand block idx back after a call on stream s has enqueued its kernels.
void scratch_give(Ctx* c, int idx, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(c->scr_mu);
    ScratchBlock& b = c->scratch[idx];
    (void)hipEventRecord(b.last, s);
    b.stream = s;
    b.taken = false;
}

// Plan, take scratch (a cached block or stream-ordered pool memory), upload,
// enqueue, hand the scratch back in stream order.
int enqueue(Ctx* c, const Params& par, int mode, uint32_t kmax, const std::vector<Req>& reqs,
            void* out_summaries, void* out_records, uint64_t* out_exceptions, uint64_t exc_cap,
            hipStream_t s)
{
    Planned P;
    int rc = plan(c, par, mode, kmax, reqs, out_exceptions != nullptr, &P);
    if (rc)
        return rc;
    char* base = nullptr;
    const int blk = scratch_take(c, P.bytes, s, &base);
    if (blk < 0) {
        hipError_t e = hipMallocFromPoolAsync((void**)&base, P.bytes, c->pool, s);
        if (e != hipSuccess || !base)
            return fail(ESQ_ENOMEM, std::string("hipMallocFromPoolAsync(scratch): ") + hipGetErrorString(e));
    }
    auto release = [&]() {
        if (blk >= 0)
            scratch_give(c, blk, s);
        else
            (void)hipFreeAsync(base, s);
    };
    bind(&P, base);
    const bool by_value = P.ivs.size() == 1;
    if (!by_value) {
        std::vector<std::pair<const void*, size_t>> parts;
        std::vector<char*> dsts;
        parts.push_back({P.ivs.data(), sizeof(Interval) * P.ivs.size()});
        dsts.push_back(base + P.o_iv);
        if (!P.items.empty()) {
            parts.push_back({P.items.data(), sizeof(uint4) * P.items.size()});
            dsts.push_back(base + P.o_items);
        }
        if ((rc = stage_upload(parts, dsts, s))) {
            release();
            return rc;
        }
    }
    rc = launch_seq(P, by_value, par.profile != 0, out_summaries, out_records, out_exceptions,
                    exc_cap, s);
    release();
    return rc;
}

int make_batch_reqs(const Ctx* c, uint32_t count, const uint64_t* lo, const uint64_t* hi,
                    uint8_t* const* d_out_mink, std::vector<Req>* reqs, bool* per_n)
{
    reqs->assign(count, Req());
    *per_n = false;
    for (uint32_t i = 0; i < count; i++) {
        if (lo[i] > hi[i])
            return fail(ESQ_EINVAL, "lo > hi in entry " + std::to_string(i));
        if (hi[i] > c->max_hi)
            return fail(ESQ_ERANGE, "hi above the max_hi given to esq_init in entry " + std::to_string(i));
        const uint64_t n0 = std::max<uint64_t>(lo[i], 3) | 1;
        const uint64_t n_odd = hi[i] > n0 ? (hi[i] - n0 + 1) / 2 : 0;
        Req& r = (*reqs)[i];
        r.I0 = (n0 - 1) / 2;
        r.I1 = r.I0 + n_odd;
        r.out_mink = d_out_mink ? d_out_mink[i] : nullptr;
        r.out_bits = nullptr;
        *per_n = *per_n || r.out_mink;
    }
    return ESQ_OK;
}

// Argument checks and the single request of esq_verify_range and its
// no-alloc variant.
int verify_range_args(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t* d_out_mink,
                      esq_summary* out_summary, uint64_t* out_exceptions, uint64_t exceptions_cap,
                      Ctx** c, Params* par, std::vector<Req>* reqs)
{
    int rc = snapshot(c, par);
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
    if (hi > (*c)->max_hi)
        return fail(ESQ_ERANGE, "hi above the max_hi given to esq_init");
    const uint64_t n0 = std::max<uint64_t>(lo, 3) | 1;
    const uint64_t n_odd = hi > n0 ? (hi - n0 + 1) / 2 : 0;
    reqs->assign(1, Req());
    Req& r = (*reqs)[0];
    r.I0 = (n0 - 1) / 2;
    r.I1 = r.I0 + n_odd;
    r.out_mink = d_out_mink;
    r.out_bits = nullptr;
    return ESQ_OK;
}

}  // namespace

// A prepared batch: planned once, scratch and descriptors resident, launched
// any number of times (directly or as a replayed hipGraph).
struct esq_batch {
    Planned P;
    char* base = nullptr;
    int device = 0;
    uint64_t generation = 0;  // Ctx::generation of the tables P.L points at
    bool profile = false;
    void* out_summaries = nullptr;
    void* out_records = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;  // private stream the kernel sequence is captured on
};

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
    // the no-alloc entry point's scratch: its address on this device, taken
    // once with the device current
    if (device >= 0 && device < kMaxDevices && !g_scratch_ptr[device]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess || !p)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = (char*)p;
    }
    bool fresh = false;
    if (!g_ctx) {
        g_ctx = new Ctx();
        g_ctx->device = device;
        g_ctx->generation = ++g_generation;
        fresh = true;
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            ncu > 0)
            g_ctx->n_cu = ncu;
        if ((e = configure_kernels()) != hipSuccess) {
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return hip_fail(e, "hipFuncSetAttribute");
        }
        // a private pool for the per-call scratch that keeps freed memory
        // (the default pool would hand it back to the driver at each
        // synchronization and map it again on the next call)
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        if ((e = hipMemPoolCreate(&g_ctx->pool, &props)) != hipSuccess) {
            g_ctx->pool = nullptr;
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return hip_fail(e, "hipMemPoolCreate");
        }
        uint64_t keep = ~0ull;
        (void)hipMemPoolSetAttribute(g_ctx->pool, hipMemPoolAttrReleaseThreshold, &keep);
        // both tables in one 2 MiB allocation (a single large page for the
        // translation caches of every CU)
        static_assert(2 * (kWheelPeriod + kWheelExtra + kWheel2Period + kWheelExtra) * 8 + kPhaseSlots * 8 <=
                          kWheelAlloc,
                      "wheel tables and phase counters exceed their allocation");
        e = hipMalloc(&g_ctx->d_wheel, kWheelAlloc);
        if (e == hipSuccess) {
            g_ctx->d_wheel2 = g_ctx->d_wheel + (kWheelPeriod + kWheelExtra);
            g_ctx->d_wheel_s = g_ctx->d_wheel2 + (kWheel2Period + kWheelExtra);
            g_ctx->d_wheel2_s = g_ctx->d_wheel_s + (kWheelPeriod + kWheelExtra);
            g_ctx->d_phase = reinterpret_cast<unsigned long long*>(g_ctx->d_wheel) + (kWheelAlloc / 8 - kPhaseSlots);
            e = hipMemset(g_ctx->d_phase, 0, kPhaseSlots * 8);
        }
        if (e != hipSuccess) {
            free_ctx(g_ctx);
            g_ctx = nullptr;
            return fail(ESQ_ENOMEM, "hipMalloc(wheel)");
        }
        if ((e = launch_wheel_build(g_ctx->d_wheel, g_ctx->d_wheel2, 0, nullptr)) != hipSuccess ||
            (e = launch_wheel_build(g_ctx->d_wheel_s, g_ctx->d_wheel2_s, 1, nullptr)) != hipSuccess) {
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
        // coarse index for the cofactor pass: idx[v] = first prime >= v * 256
        const uint32_t pidx_n = (uint32_t)((need >> kPidxShift) + 3);
        std::vector<uint32_t> idx(pidx_n);
        for (uint32_t v = 0, i = 0; v < pidx_n; v++) {
            const uint64_t bound = (uint64_t)v << kPidxShift;
            while (i < pr.size() && pr[i] < bound)
                i++;
            idx[v] = i;
        }
        // Barrett reciprocals floor(2^64 / p^2) of the primes the large-prime
        // pass reduces by (p <= kCofactorPrime), 8-byte aligned after the index
        const size_t n_main = pr.size();
        const uint32_t n_qinv = (uint32_t)(std::upper_bound(pr.begin(), pr.end(),
                                                            (uint32_t)kCofactorPrime) - pr.begin());
        pr.insert(pr.end(), idx.begin(), idx.end());
        if (pr.size() & 1)
            pr.push_back(0);
        const size_t qinv_at = pr.size();  // in uint32 units
        for (uint32_t i = 0; i < n_qinv; i++) {
            const uint64_t q = (uint64_t)pr[i] * pr[i];
            const uint64_t m = (uint64_t)(((unsigned __int128)1 << 64) / q);
            pr.push_back((uint32_t)m);
            pr.push_back((uint32_t)(m >> 32));
        }
        uint32_t* d = nullptr;
        e = hipMalloc(&d, pr.size() * 4);
        if (e != hipSuccess)
            return fail(ESQ_ENOMEM, "hipMalloc(primes)");
        if ((e = hipMemcpy(d, pr.data(), pr.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(e, "hipMemcpy(primes)");
        }
        pr.resize(n_main);
        c->qinv_at = qinv_at;
        c->n_qinv = n_qinv;
        if (c->d_primes) {
            (void)hipDeviceSynchronize();
            (void)hipFree(c->d_primes);
        }
        c->d_primes = d;
        c->pidx_n = pidx_n;
        c->primes.swap(pr);
        c->inv_pref.swap(pref);
        c->plimit = need;
        c->generation = ++g_generation;  // prepared batches hold the old table
    }
    c->max_hi = std::max(c->max_hi, max_hi);
    // the medium-prime tables of the current knobs (they need the primes)
    int rc = prebuild_med_table(c, g_par);
    if (rc)
        return rc;
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
    if (!d_bits)
        return fail(ESQ_EINVAL, "d_bits is null");
    const uint64_t n_bits = (hi - m0 + 1) / 2;
    const uint64_t I0 = (m0 - 1) / 2;
    std::vector<Req> reqs(1);
    reqs[0].I0 = I0;
    reqs[0].I1 = I0 + n_bits;
    reqs[0].out_mink = nullptr;
    reqs[0].out_bits = d_bits;
    return enqueue(c, par, 2, 0, reqs, nullptr, nullptr, nullptr, 0, (hipStream_t)stream);
}

int esq_verify_range(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t* d_out_mink,
                     esq_summary* out_summary, esq_record* out_records, uint64_t* out_exceptions,
                     uint64_t exceptions_cap, void* stream)
{
    t_err.clear();
    Ctx* c;
    Params par;
    std::vector<Req> reqs;
    int rc = verify_range_args(lo, hi, kmax, d_out_mink, out_summary, out_exceptions,
                               exceptions_cap, &c, &par, &reqs);
    if (rc)
        return rc;
    return enqueue(c, par, d_out_mink ? 1 : 0, kmax, reqs, out_summary, out_records,
                   exceptions_cap ? out_exceptions : nullptr, exceptions_cap, (hipStream_t)stream);
}

int esq_verify_range_noalloc(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t* d_out_mink,
                             esq_summary* out_summary, esq_record* out_records,
                             uint64_t* out_exceptions, uint64_t exceptions_cap, void* stream)
{
    t_err.clear();
    Ctx* c;
    Params par;
    std::vector<Req> reqs;
    int rc = verify_range_args(lo, hi, kmax, d_out_mink, out_summary, out_exceptions,
                               exceptions_cap, &c, &par, &reqs);
    if (rc)
        return rc;
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (c->device >= 0 && c->device < kMaxDevices)
            base = g_scratch_ptr[c->device];
    }
    if (!base)
        return fail(ESQ_ENOINIT, "no static scratch on this device (device index above 63)");
    Planned P;
    const bool exc_list = exceptions_cap != 0;
    if ((rc = plan(c, par, d_out_mink ? 1 : 0, kmax, reqs, exc_list, &P, true)))
        return rc;
    if (P.bytes > ESQ_NOALLOC_SCRATCH_MAX)
        return fail(ESQ_ERANGE, "interval needs " + std::to_string(P.bytes) +
                                    " bytes of scratch, above the static " +
                                    std::to_string(ESQ_NOALLOC_SCRATCH_MAX) +
                                    " (ESQ_NOALLOC_SCRATCH_MAX)");
    bind(&P, base);
    // the single interval's descriptor travels as a kernel argument: no
    // upload, no staging buffer; no profiling events either
    return launch_seq(P, true, false, out_summary, out_records,
                      exc_list ? out_exceptions : nullptr, exceptions_cap, (hipStream_t)stream);
}

int esq_verify_batch(uint32_t count, const uint64_t* lo, const uint64_t* hi, uint32_t kmax,
                     uint8_t* const* d_out_mink, esq_summary* out_summaries,
                     esq_record* out_records, void* stream)
{
    t_err.clear();
    Ctx* c;
    Params par;
    int rc = snapshot(&c, &par);
    if (rc)
        return rc;
    if (count == 0)
        return ESQ_OK;
    if (!lo || !hi || !out_summaries)
        return fail(ESQ_EINVAL, "null lo, hi or out_summaries");
    if (kmax > 63)
        return fail(ESQ_EINVAL, "kmax > 63");
    std::vector<Req> reqs;
    bool per_n = false;
    if ((rc = make_batch_reqs(c, count, lo, hi, d_out_mink, &reqs, &per_n)))
        return rc;
    return enqueue(c, par, per_n ? 1 : 0, kmax, reqs, out_summaries, out_records, nullptr, 0,
                   (hipStream_t)stream);
}

int esq_scratch_bytes(uint32_t count, const uint64_t* lo, const uint64_t* hi, uint32_t kmax,
                      uint64_t* out_bytes)
{
    t_err.clear();
    if (!out_bytes)
        return fail(ESQ_EINVAL, "out_bytes is null");
    *out_bytes = 0;
    Ctx* c;
    Params par;
    int rc = snapshot(&c, &par);
    if (rc)
        return rc;
    if (count == 0)
        return ESQ_OK;
    if (!lo || !hi)
        return fail(ESQ_EINVAL, "null lo or hi");
    if (kmax > 63)
        return fail(ESQ_EINVAL, "kmax > 63");
    std::vector<Req> reqs;
    bool per_n = false;
    if ((rc = make_batch_reqs(c, count, lo, hi, nullptr, &reqs, &per_n)))
        return rc;
    Planned P;
    if ((rc = plan(c, par, 0, kmax, reqs, false, &P)))
        return rc;
    *out_bytes = P.bytes;
    return ESQ_OK;
}

int esq_batch_create(uint32_t count, const uint64_t* lo, const uint64_t* hi, uint32_t kmax,
                     uint8_t* const* d_out_mink, esq_summary* out_summaries,
                     esq_record* out_records, esq_batch** out_handle)
{
    t_err.clear();
    if (!out_handle)
        return fail(ESQ_EINVAL, "out_handle is null");
    *out_handle = nullptr;
    Ctx* c;
    Params par;
    int rc = snapshot(&c, &par);
    if (rc)
        return rc;
    if (count == 0 || !lo || !hi || !out_summaries)
        return fail(ESQ_EINVAL, "empty batch or null lo, hi, out_summaries");
    if (kmax > 63)
        return fail(ESQ_EINVAL, "kmax > 63");
    std::vector<Req> reqs;
    bool per_n = false;
    if ((rc = make_batch_reqs(c, count, lo, hi, d_out_mink, &reqs, &per_n)))
        return rc;
    esq_batch* b = new esq_batch();
    b->device = c->device;
    b->profile = par.profile != 0;
    b->out_summaries = out_summaries;
    b->out_records = out_records;
    b->generation = c->generation;
    if ((rc = plan(c, par, per_n ? 1 : 0, kmax, reqs, false, &b->P))) {
        delete b;
        return rc;
    }
    hipError_t e = hipMalloc((void**)&b->base, b->P.bytes);
    if (e != hipSuccess) {
        delete b;
        return fail(ESQ_ENOMEM, "hipMalloc(batch scratch)");
    }
    bind(&b->P, b->base);
    if ((e = hipMemcpy(b->base + b->P.o_iv, b->P.ivs.data(), sizeof(Interval) * b->P.ivs.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (!b->P.items.empty() &&
         (e = hipMemcpy(b->base + b->P.o_items, b->P.items.data(),
                        sizeof(uint4) * b->P.items.size(), hipMemcpyHostToDevice)) != hipSuccess)) {
        (void)hipFree(b->base);
        delete b;
        return hip_fail(e, "hipMemcpy(batch descriptors)");
    }
    *out_handle = b;
    return ESQ_OK;
}

int esq_batch_launch(esq_batch* b, int use_graph, void* stream)
{
    t_err.clear();
    if (!b)
        return fail(ESQ_EINVAL, "null batch");
    {
        // the batch's launch points at the context's prime, wheel and
        // medium-prime tables: they must still be the ones it was planned on
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ctx || g_ctx->device != b->device || g_ctx->generation != b->generation)
            return fail(ESQ_EINVAL, "prepared batch is stale: esq_init or esq_shutdown has replaced "
                                    "the tables it was planned on (destroy it and create it again)");
    }
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess)
        return hip_fail(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph)
        return launch_seq(b->P, false, b->profile, b->out_summaries, b->out_records, nullptr, 0, s);
    if (!b->exec) {
        // capture on a private stream (the legacy default stream cannot be
        // captured); the instantiated graph is launched on the caller's stream
        if (!b->capture &&
            (e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate(capture)");
        if ((e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        int rc = launch_seq(b->P, false, false, b->out_summaries, b->out_records, nullptr, 0,
                            b->capture);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->capture, &g);
        if (rc) {
            if (g)
                (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamEndCapture");
        if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->graph = g;
    }
    if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess)
        return hip_fail(e, "hipGraphLaunch");
    return ESQ_OK;
}

void esq_batch_destroy(esq_batch* b)
{
    if (!b)
        return;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->capture)
        (void)hipStreamDestroy(b->capture);
    if (b->base)
        (void)hipFree(b->base);
    delete b;
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
    } else if (n == "sieve_seg_log2") {
        if (value < kMinSegLog2 || value > kMaxSegLog2)
            return fail(ESQ_EINVAL, "sieve_seg_log2 out of range");
        g_par.sieve_seg_log2 = (int)value;
    } else if (n == "kh") {
        if (value < 1 || value > kMaxKh)
            return fail(ESQ_EINVAL, "kh out of range");
        g_par.kh = (int)value;
    } else if (n == "block" || n == "per_n_block" || n == "sieve_block") {
        if (value < 64 || value > 1024 || value % 64)
            return fail(ESQ_EINVAL, n + " out of range");
        (n == "block" ? g_par.block : n == "per_n_block" ? g_par.per_n_block : g_par.sieve_block) = (int)value;
    } else if (n == "entry_hits") {
        if (value < 1 || value > 4096)
            return fail(ESQ_EINVAL, "entry_hits out of range");
        g_par.entry_hits = (int)value;
    } else if (n == "tail_cap") {
        if (value < 1 || value > (int64_t)1 << 30)
            return fail(ESQ_EINVAL, "tail_cap out of range");
        g_par.tail_cap = value;
    } else if (n == "phase_clock") {
        if (value < 0 || value > 1)
            return fail(ESQ_EINVAL, "phase_clock must be 0 or 1");
        g_par.phase_clock = (int)value;
    } else if (n == "profile") {
        if (value < 0 || value > 1)
            return fail(ESQ_EINVAL, "profile must be 0 or 1");
        g_par.profile = (int)value;
    } else if (n == "medium_max") {
        if (value < 11 || value > 11000)
            return fail(ESQ_EINVAL, "medium_max out of range");
        g_par.medium_max = value;
    } else if (n == "bucket_cap") {
        if (value < 0 || value > 4096)
            return fail(ESQ_EINVAL, "bucket_cap out of range");
        g_par.bucket_cap = value;
    } else if (n == "items_per_wg") {
        if (value < 1 || value > 1024)
            return fail(ESQ_EINVAL, "items_per_wg out of range");
        g_par.items_per_wg = value;
    } else if (n == "runs_per_wg") {
        if (value < 1 || value > 64)
            return fail(ESQ_EINVAL, "runs_per_wg out of range");
        g_par.runs_per_wg = value;
    } else if (n == "stagger") {
        if (value < 0 || value > 4096)
            return fail(ESQ_EINVAL, "stagger out of range");
        g_par.stagger = value;
    } else if (n == "cof_weight") {
        if (value < 1 || value > 10000)
            return fail(ESQ_EINVAL, "cof_weight out of range");
        g_par.cof_weight = value;
    } else if (n == "priority") {
        if (value < 0 || value > 1)
            return fail(ESQ_EINVAL, "priority must be 0 or 1");
        g_par.priority = value;
    } else {
        return fail(ESQ_EINVAL, "unknown parameter " + n);
    }
    if (g_ctx && (n == "seg_log2" || n == "kh" || n == "medium_max" || n == "entry_hits" ||
                  n == "block" || n == "per_n_block")) {
        hipError_t e = hipSetDevice(g_ctx->device);
        if (e != hipSuccess)
            return hip_fail(e, "hipSetDevice");
        return prebuild_med_table(g_ctx, g_par);
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
    if (n == "sieve_seg_log2") return g_par.sieve_seg_log2;
    if (n == "kh") return g_par.kh;
    if (n == "block") return g_par.block;
    if (n == "per_n_block") return g_par.per_n_block;
    if (n == "sieve_block") return g_par.sieve_block;
    if (n == "entry_hits") return g_par.entry_hits;
    if (n == "tail_cap") return g_par.tail_cap;
    if (n == "profile") return g_par.profile;
    if (n == "phase_clock") return g_par.phase_clock;
    if (n == "medium_max") return g_par.medium_max;
    if (n == "bucket_cap") return g_par.bucket_cap;
    if (n == "items_per_wg") return g_par.items_per_wg;
    if (n == "runs_per_wg") return g_par.runs_per_wg;
    if (n == "stagger") return g_par.stagger;
    if (n == "priority") return g_par.priority;
    if (n == "cof_weight") return g_par.cof_weight;
    return -1;
}

int esq_phase_take(uint64_t* ticks)
{
    t_err.clear();
    if (!ticks)
        return fail(ESQ_EINVAL, "null pointer");
    Ctx* c = g_ctx;
    if (!c)
        return fail(ESQ_ENOINIT, "esq_init has not been called");
    hipError_t e;
    if ((e = hipSetDevice(c->device)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess ||
        (e = hipMemcpy(ticks, c->d_phase, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemset(c->d_phase, 0, kPhaseSlots * 8)) != hipSuccess)
        return hip_fail(e, "phase counters");
    return ESQ_OK;
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
    std::lock_guard<std::mutex> sl(g_stage_mu);
    for (auto& st : g_stage) {
        (void)hipHostFree(st.host);
        (void)hipEventDestroy(st.done);
    }
    g_stage.clear();
}

}  // extern "C"
