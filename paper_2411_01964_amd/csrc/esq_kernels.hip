// HIP kernels for gfx950 (wave64).  Exact integer work only: no floating
// point on any result and no matrix cores -- the sieve and the search are bit
// operations over 64-bit words.
//
//   k_wheel_build  periodic patterns of odd multiples of 9, 25, 49 and of 121, 169 (once)
//   k_prepare      zero the per-launch accumulators and the work queue
//   k_bucket       primes above the medium range: every odd multiple of p^2
//                  that falls in a segment region goes to that segment's hit
//                  slots (by first hit up to a cut-over chosen per launch, at
//                  most 2^20; by cofactor enumeration above it)
//   k_verify       persistent workgroups pull runs of consecutive segments;
//                  per segment: Algorithm 1 in LDS, then Algorithm 2 as a
//                  bit-sliced scan of the LDS bitmap (in per-n mode also one
//                  byte per n to HBM, staged through LDS; in sieve mode the
//                  bitmap itself to HBM)
//   k_tail         exact search for the rare n not resolved from LDS
//   k_finalize     per interval: aggregates, record-setters, exceptions
#include <type_traits>

#include "esq.h"
#include "esq_internal.h"

namespace esq {

// ------------------------------------------------------------ wheel table

// Word w holds bits for odd indices 64w .. 64w+63 (mod the period).  An odd
// index x is an odd multiple of q = p^2 iff x = (q - 1)/2 (mod q).  A word
// pattern repeats every `period` words when gcd(64, period) = 1: 9 * 25 * 49
// for the first table, 121 * 169 for the second.  Both tables carry
// kWheelExtra more words so that a region never wraps; together they take
// about 0.5 MB and stay in L2.  A second pair of tables holds the same
// patterns one position lower (word w: odd indices 64w - 1 .. 64w + 62), for
// the search's regions, whose bit 0 sits one position below a word boundary.
__global__ void k_wheel_build(uint64_t* wheel, uint64_t* wheel2, uint32_t shift)
{
    const uint32_t n1 = kWheelPeriod + kWheelExtra, n2 = kWheel2Period + kWheelExtra;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < n1 + n2;
         w += gridDim.x * blockDim.x) {
        const bool second = w >= n1;
        const uint32_t ww = second ? w - n1 : w;
        const uint32_t period = second ? kWheel2Period : kWheelPeriod;
        const uint32_t base = (uint32_t)(((uint64_t)ww * 64u + period - shift) % period);
        uint64_t word = 0;
        for (uint32_t b = 0; b < 64; b++) {
            const uint32_t x = base + b;
            const bool hit = second ? (x % 121u == 60u || x % 169u == 84u)
                                    : (x % 9u == 4u || x % 25u == 12u || x % 49u == 24u);
            if (hit)
                word |= 1ull << b;
        }
        if (second)
            wheel2[ww] = word;
        else
            wheel[ww] = word;
    }
}

hipError_t launch_wheel_build(uint64_t* wheel, uint64_t* wheel2, uint32_t shift, hipStream_t s)
{
    hipLaunchKernelGGL(k_wheel_build, dim3(1024), dim3(256), 0, s, wheel, wheel2, shift);
    return hipGetLastError();
}

typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Output pointers read from an Interval in memory are generic: stores through
// them become flat stores, which also count on the LDS wait counter, so every
// later wait for an LDS read would wait for the stores to reach memory too.
// Stores to the output buffers go through these global-space views instead.
typedef __attribute__((address_space(1))) uint8_t g_u8;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;
typedef __attribute__((address_space(1))) u64x2 g_u64x2;
typedef __attribute__((address_space(1))) unsigned long long g_ull;
typedef __attribute__((address_space(1))) unsigned int g_uint;
__device__ __forceinline__ void g_add(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_fetch_add((g_ull*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_min(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_fetch_min((g_ull*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_or(unsigned int* p, unsigned int v)
{
    __hip_atomic_fetch_or((g_uint*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// popcount(x) + acc in one v_bcnt_u32_b32
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// --------------------------------------------------------------- prepare

__global__ void k_prepare(Launch L, Acc* accs, Interval iv0, int write_iv0, uint32_t nseg_total)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    if (write_iv0 && t == 0)
        *const_cast<Interval*>(L.iv) = iv0;
    for (uint32_t i = t; i < L.n_iv * 65u; i += stride) {
        Acc* a = accs + i / 65u;
        const uint32_t k = i % 65u;
        if (k < 16)
            a->cnt[k] = 0;
        a->first[k] = kNone;
        a->deep_hist[k] = 0;
        if (k == 0) {
            a->tail_count = 0;
            a->status = 0;
            a->pad = 0;
        }
    }
    if (L.bucket_cnt)
        for (uint32_t i = t; i < nseg_total; i += stride)
            L.bucket_cnt[i] = 0;
    if (t == 0) {
        *L.queue = 0;
        *L.tail_count = 0;
    }
}

hipError_t launch_prepare(const Launch& L, Acc* accs, const Interval* iv_single,
                          uint32_t nseg_total, hipStream_t s)
{
    Interval iv0;
    __builtin_memset(&iv0, 0, sizeof(iv0));
    if (iv_single)
        iv0 = *iv_single;
    hipLaunchKernelGGL(k_prepare, dim3(256), dim3(256), 0, s, L, accs, iv0, iv_single ? 1 : 0,
                       nseg_total);
    return hipGetLastError();
}

// ------------------------------------------------------- large primes

// least y >= 0 with B0 + y an odd multiple of q, in odd-index terms
__device__ __forceinline__ uint64_t first_hit(int64_t B0, uint64_t q)
{
    const int64_t d = (int64_t)((q - 1) >> 1) - B0;
    int64_t f = d % (int64_t)q;
    if (f < 0)
        f += (int64_t)q;
    return (uint64_t)f;
}

// x mod q for any x < 2^64 by Barrett reduction (Barrett, CRYPTO '86): with
// m = floor(2^64 / q), t = floor(x m / 2^64) is floor(x / q) or one less, so
// x - t q lies in [0, 2q) and one conditional subtraction finishes it
__device__ __forceinline__ uint64_t mod_barrett(uint64_t x, uint64_t q, uint64_t m)
{
    const uint64_t r = x - __umul64hi(x, m) * q;
    return r >= q ? r - q : r;
}

// first_hit with the prime's Barrett reciprocal m = floor(2^64 / q)
__device__ __forceinline__ uint64_t first_hit_b(int64_t B0, uint64_t q, uint64_t m)
{
    const int64_t h = (int64_t)((q - 1) >> 1);
    if (B0 <= h)
        return mod_barrett((uint64_t)(h - B0), q, m);
    const uint64_t r = mod_barrett((uint64_t)(B0 - h), q, m);
    return r ? q - r : 0;
}

__device__ __forceinline__ uint64_t isqrt_floor(uint64_t x)
{
    uint64_t r = (uint64_t)sqrt((double)x);
    while (r > 0 && r * r > x)
        r--;
    while ((r + 1) * (r + 1) <= x)
        r++;
    return r;
}

// Segment s of an interval covers region offsets y in [s S, s S + R): a hit
// belongs to segment floor(y / S) and to each earlier segment still reaching it.
__device__ __forceinline__ void bucket_emit(const Launch& L, const Interval& iv, uint64_t y)
{
    const uint64_t S = 1ull << L.log2S;
    const uint64_t R = (uint64_t)L.rw * 64;
    uint64_t seg = y >> L.log2S;
    uint64_t off = y & (S - 1);
    while (off < R) {
        if (seg < iv.nseg) {
            const uint32_t gs = iv.seg_base + (uint32_t)seg;
            const uint32_t pos = atomicAdd(&L.bucket_cnt[gs], 1u);
            if (pos < L.bucket_cap)
                L.bucket_slot[(uint64_t)gs * L.bucket_cap + pos] = (uint32_t)off;
        }
        if (seg == 0)
            break;
        seg--;
        off += S;
    }
}

// grid.y = interval.  Work units, in order: kHeavyLanes-wide groups of lanes
// for each of the first n_heavy bucket primes (many hits: the group strides
// over them), then one thread per remaining prime of the direct range
// primes[med_end, b_direct_end), then, for the primes above it, kCofactorLanes
// lanes for each of the first n_cof_wide odd cofactors j (wide ranges) and one
// thread for each remaining j.
constexpr uint32_t kHeavyLanes = 64;
constexpr uint32_t kCofactorLanes = 8;

__global__ __launch_bounds__(256) void k_bucket(Launch L, uint32_t n_heavy, uint32_t max_direct)
{
    const Interval iv = L.iv[blockIdx.y];
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t B0 = iv.A0 - (int64_t)L.hlo_words * 64 - (int64_t)L.origin;  // region bit 0
    const uint64_t S = 1ull << L.log2S;
    const uint64_t E = (uint64_t)(iv.nseg ? iv.nseg - 1 : 0) * S + (uint64_t)L.rw * 64;
    if (iv.nseg == 0)
        return;
    const uint64_t heavy_units = (uint64_t)n_heavy * kHeavyLanes;
    if (t < heavy_units) {
        const uint64_t pi = L.med_end + t / kHeavyLanes;
        const uint32_t g = (uint32_t)(t % kHeavyLanes);
        if (pi >= iv.b_direct_end)
            return;
        const uint64_t p = L.primes[pi];
        const uint64_t q = p * p;
        const uint64_t f = pi < L.n_qinv ? first_hit_b(B0, q, L.qinv[pi]) : first_hit(B0, q);
        for (uint64_t y = f + g * q; y < E; y += kHeavyLanes * q)
            bucket_emit(L, iv, y);
        return;
    }
    const uint64_t td = t - heavy_units;
    if (td < max_direct) {
        const uint64_t pi = L.med_end + n_heavy + td;
        if (pi >= iv.b_direct_end)
            return;
        const uint64_t p = L.primes[pi];
        const uint64_t q = p * p;
        const uint64_t f = pi < L.n_qinv ? first_hit_b(B0, q, L.qinv[pi]) : first_hit(B0, q);
        for (uint64_t y = f; y < E; y += q)
            bucket_emit(L, iv, y);
        return;
    }
    // odd multiples j p^2 of the primes above the direct range, one thread
    // per odd cofactor j: the p with j p^2 in [m_lo, m_hi] form one range,
    // empty for most j when the interval is short
    const uint64_t tc = td - max_direct;
    const uint64_t wide_threads = (uint64_t)iv.n_cof_wide * kCofactorLanes;
    uint64_t c;
    uint32_t g = 0, lanes = 1;
    if (tc < wide_threads) {
        c = tc / kCofactorLanes;
        g = (uint32_t)(tc % kCofactorLanes);
        lanes = kCofactorLanes;
    } else {
        c = iv.n_cof_wide + (tc - wide_threads);
    }
    if (c >= iv.n_cof || iv.b_direct_end >= iv.pmax_end)
        return;
    const uint64_t j = 2 * c + 1;
    const uint64_t m_lo = B0 > 0 ? 2 * (uint64_t)B0 + 1 : 1;
    const uint64_t m_hi = 2 * (uint64_t)(B0 + (int64_t)E - 1) + 1;
    // least pa with j pa^2 >= m_lo and largest pb with j pb^2 <= m_hi: a
    // double estimate (within one of the answer), then exact corrections
    uint64_t pa = (uint64_t)sqrt((double)m_lo / (double)j);
    while (pa > 0 && j * pa * pa >= m_lo)
        pa--;
    while (j * pa * pa < m_lo)
        pa++;
    uint64_t pb = (uint64_t)sqrt((double)m_hi / (double)j) + 1;
    while (j * pb * pb > m_hi)
        pb--;
    if (pa > pb || pb < (uint64_t)L.primes[iv.b_direct_end])
        return;
    // first prime >= pa among primes[b_direct_end, pmax_end): the coarse
    // index narrows the search to one 256-wide stretch of integers
    const uint64_t v = min(pa >> kPidxShift, (uint64_t)L.pidx_n - 2);
    uint32_t lo = L.pidx[v], hi = L.pidx[v + 1];
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)L.primes[mid] < pa)
            lo = mid + 1;
        else
            hi = mid;
    }
    lo = max(lo, iv.b_direct_end);
    for (uint32_t i = lo + g; i < iv.pmax_end; i += lanes) {
        const uint64_t p = L.primes[i];
        if (p > pb)
            break;
        bucket_emit(L, iv, (j * p * p - 1) / 2 - (uint64_t)B0);
    }
}

hipError_t launch_bucket(const Launch& L, uint32_t n_heavy, uint32_t max_direct, uint32_t max_cof,
                         hipStream_t s)
{
    const uint64_t threads = (uint64_t)n_heavy * kHeavyLanes + max_direct + (uint64_t)max_cof;
    if (threads == 0 || L.n_iv == 0)
        return hipSuccess;
    const uint32_t bx = (uint32_t)((threads + 255) / 256);
    hipLaunchKernelGGL(k_bucket, dim3(bx, L.n_iv), dim3(256), 0, s, L, n_heavy, max_direct);
    return hipGetLastError();
}

// ------------------------------------------------------- segment kernel

// 4 bits -> 4 bytes holding 0 or 1
__device__ __forceinline__ uint32_t spread4(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }

// bits of the 64 n-indices j0 .. j0+63 that lie in [I0, I1)
__device__ __forceinline__ uint64_t valid_mask(uint64_t j0, uint64_t I0, uint64_t I1)
{
    if (j0 + 64 <= I0 || j0 >= I1)
        return 0;
    uint64_t m = ~0ull;
    if (I0 > j0)
        m &= ~0ull << (I0 - j0);
    if (I1 < j0 + 64)
        m &= ~0ull >> (j0 + 64 - I1);
    return m;
}

// Store the 64 depth bytes D (4 per dword) of one word at out[0..63], only
// where V has a bit.  Interior dwords that are wholly ours and valid go out
// as aligned 32-bit stores; the rest byte by byte.
__device__ __forceinline__ void store_depths(g_u8* out, const uint32_t (&D)[16], uint64_t V)
{
    // whole word, 16-byte aligned (every word of an interval whose first
    // n-index is a multiple of 16): four 16-byte stores
    if (V == ~0ull && ((uintptr_t)out & 15u) == 0) {
        g_u32x4* o = (g_u32x4*)out;
#pragma unroll
        for (int q = 0; q < 4; q++)
            o[q] = u32x4{D[4 * q], D[4 * q + 1], D[4 * q + 2], D[4 * q + 3]};
        return;
    }
    const uint32_t mis = (uint32_t)((uintptr_t)out & 3u);
    g_u8* al = out - mis;
#pragma unroll
    for (int t = 0; t <= 16; t++) {
        // the aligned dword at al + 4t holds stream bytes 4t - mis .. 4t - mis + 3
        const uint32_t lo = t > 0 ? D[t - 1] : 0u;
        const uint32_t hi = t < 16 ? D[t] : 0u;
        const uint32_t val = mis ? ((hi << (8 * mis)) | (lo >> (32 - 8 * mis))) : hi;
        const int b0 = 4 * t - (int)mis;
        bool all = true;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int b = b0 + i;
            all = all && b >= 0 && b < 64 && ((V >> (b & 63)) & 1ull);
        }
        if (all) {
            *(g_u32*)(al + 4 * t) = val;
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int b = b0 + i;
                if (b >= 0 && b < 64 && ((V >> (b & 63)) & 1ull))
                    al[4 * t + i] = (uint8_t)(val >> (8 * i));
            }
        }
    }
}

__device__ __forceinline__ void mark(uint32_t* bm32, uint32_t pos)
{
    // the byte address of the word as (pos >> 3) & ~3: one shift (a half-rate
    // operation on this chip, like the mask's) and one full-rate AND, where
    // (pos >> 5) << 2 would take two shifts
    // The bitmap starts at LDS address 0 (the kernel has no static LDS), so
    // the byte offset is the LDS address itself.
    (void)bm32;
    uint32_t a;
    asm("v_lshrrev_b32 %0, 3, %1" : "=v"(a) : "v"(pos));
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    lds_u32* w = (lds_u32*)(uintptr_t)(a & ~3u);
    __hip_atomic_fetch_or(w, 1u << (pos & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Store bytes [b0, b1) of the 16 bytes v at the 16-byte aligned p (b0, b1
// wave-uniform): whole dwords as dwords, the rest byte by byte.
__device__ __forceinline__ void store_part16(g_u8* p, const u32x4 v, uint32_t b0, uint32_t b1)
{
#pragma unroll
    for (uint32_t t = 0; t < 4; t++) {
        if (4 * t >= b0 && 4 * t + 4 <= b1) {
            *(g_u32*)(p + 4 * t) = v[t];
        } else {
#pragma unroll
            for (uint32_t j = 0; j < 4; j++)
                if (4 * t + j >= b0 && 4 * t + j < b1)
                    p[4 * t + j] = (uint8_t)(v[t] >> (8 * j));
        }
    }
}

// Position of 16-byte slot s (-4 <= s < 260) in a staging area: the 4 slots
// of word w = s/4 are rotated by (w/2 xor w/8) mod 4, so that any 8 (or 16)
// consecutive lanes writing one slot of their words, or reading consecutive
// slots, touch distinct groups of LDS banks, with 32 or with 64 banks.
__device__ __forceinline__ int stage_pos(int s)
{
    const int w = s >> 2;
    return 4 * w + (((s & 3) + ((w >> 1) ^ (w >> 3))) & 3);
}

// The 16 output bytes of aligned chunk c, which begins delta bytes before
// staged slot c, from the slots A = c - 1 and B = c: x holds the five dwords
// that start KQ = ceil(delta / 4) dwords before slot c, and each output dword
// is the window of two neighbours that starts sh = (-delta) mod 4 bytes in.
template <int KQ>
__device__ __forceinline__ u32x4 stage_shift(const u32x4 A, const u32x4 B, uint32_t sh)
{
    uint32_t x[5];
#pragma unroll
    for (int i = 0; i < 5; i++)
        x[i] = i < KQ ? A[4 + i - KQ] : B[(i - KQ) & 3];
    return u32x4{__builtin_amdgcn_alignbyte(x[1], x[0], sh), __builtin_amdgcn_alignbyte(x[2], x[1], sh),
                 __builtin_amdgcn_alignbyte(x[3], x[2], sh), __builtin_amdgcn_alignbyte(x[4], x[3], sh)};
}

// Per-n mode: write a wave's 4096 depth bytes (lane l holds bytes 64l ..
// 64l+63 of the run in D) to out .. out+4095 through the wave's staging area
// st (slot 0; 4 guard slots on either side), so that each global store
// writes 1 KB of consecutive bytes.  The run starts delta = out mod 16 bytes
// past an aligned chunk; the first and last chunks, shared with the
// neighbouring runs, are written in part.
template <int KQ>
__device__ __forceinline__ void stage_store_run(u32x4* st, g_u8* out, const uint32_t (&D)[16],
                                                uint32_t lane, uint32_t delta)
{
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 4; q++)
        st[stage_pos(4 * (int)lane + q)] = u32x4{D[4 * q], D[4 * q + 1], D[4 * q + 2], D[4 * q + 3]};
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    g_u8* g = out - delta;  // 16-byte aligned
    g_u32x4* go = (g_u32x4*)g;
    const uint32_t sh = (0u - delta) & 3u;
    u32x4 last;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int c = 64 * r + (int)lane;
        const u32x4 B = st[stage_pos(c)];
        if (KQ == 0) {
            go[c] = B;
            continue;
        }
        const u32x4 v = stage_shift<KQ>(st[stage_pos(c - 1)], B, sh);
        if (r == 0 && lane == 0)
            store_part16(g, v, delta, 16);
        else
            go[c] = v;
        last = B;
    }
    if (KQ != 0 && lane == 63)
        store_part16(g + 4096, stage_shift<KQ>(last, last, sh), 0, delta);
}

// LDS layout of k_verify: the region bitmap (rw words), a control block of
// kVerifyCtrlWords words (per-item first-n slots, level counts, the item,
// phase-clock sums), then the medium primes' (q, S mod q), their current
// first-hit offsets, the lane-task table when it fits, and in per-n mode
// (when it fits) one store-staging area per wave, 16-byte aligned.
__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// MODE 0: verify, aggregates only; MODE 1: verify + per-n bytes;
// MODE 2: Algorithm 1 alone, bitmap to HBM.  PH: the phase-clock instance
// (measurement only).
template <int MODE, bool PH = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 8 : 4))) void k_verify(Launch L)
{
    // No static LDS: the bitmap sits at LDS address 0, so a bit position
    // turns into a word address without a base offset.
    extern __shared__ uint64_t lds[];

    const uint32_t tid = threadIdx.x, T = blockDim.x, lane = tid & 63u;
    const uint32_t S = 1u << L.log2S, SW = S >> 6;
    const uint32_t R = L.rw * 64;
    const uint32_t HW = L.hlo_words;
    const uint32_t nmed = L.med_end - kFirstMedium;
    const uint32_t klds = L.k_lds;
    const uint32_t wstep = SW % kWheelPeriod;
    uint64_t* bm = lds;
    uint32_t* bm32 = reinterpret_cast<uint32_t*>(bm);
    constexpr uint32_t kCntAt = kMaxKh + 2, kItemAt = kCntAt + (kMaxKh + 2) / 2, kPhAt = kItemAt + 2;
    static_assert(kPhAt + 3 <= kVerifyCtrlWords, "k_verify control block");
    unsigned long long* s_first = reinterpret_cast<unsigned long long*>(lds + L.rw);  // kMaxKh + 2
    uint32_t* s_cnt = reinterpret_cast<uint32_t*>(lds + L.rw + kCntAt);               // kMaxKh + 1
    uint32_t* s_item = reinterpret_cast<uint32_t*>(lds + L.rw + kItemAt);             // 4
    unsigned long long* s_ph = reinterpret_cast<unsigned long long*>(lds + L.rw + kPhAt);  // 3 (phase clock)
    uint2* s_medq = reinterpret_cast<uint2*>(lds + L.rw + kVerifyCtrlWords);
    uint32_t* s_f = reinterpret_cast<uint32_t*>(s_medq + nmed);
    uint2* s_task = reinterpret_cast<uint2*>(lds + L.rw + kVerifyCtrlWords + nmed + (nmed + 1) / 2);
    // per-n mode: this wave's 4 KB staging area for the depth bytes
    u32x4* s_stage = reinterpret_cast<u32x4*>(lds + verify_stage_word(L.rw, nmed, L.tasks_in_lds ? L.n_tasks : 0u)) +
                     (tid >> 6) * (kStageWordsPerWave / 2) + 4;

    // per-launch tables into LDS (the bitmap region is rewritten per segment)
    for (uint32_t i = tid; i < nmed; i += T)
        s_medq[i] = L.medq[i];
    if (L.tasks_in_lds)
        for (uint32_t i = tid; i < L.n_tasks; i += T)
            s_task[i] = L.tasks[i];

    // per-lane counts of levels 1 .. kRegLevels; deeper levels, reached by few
    // words, count straight into s_cnt
    constexpr int kRegLevels = 5;
    uint32_t cnt[kRegLevels + 1];
    uint32_t found = 0;       // levels whose least n this wave has already offered
    uint32_t cur_iv = ~0u;    // interval of the partial totals (~0: none)
    uint32_t acc_segs = 0;    // segments in the partial totals
    auto flush = [&](uint32_t iv) {
        if (MODE != 2) {
            Acc* acc = L.iv[iv].acc;
#pragma unroll
            for (int k = 1; k <= kRegLevels; k++) {
                if (k > (int)klds)
                    break;
                uint32_t v = cnt[k];
                for (int o = 32; o > 0; o >>= 1)
                    v += __shfl_xor(v, o);
                if (lane == 0 && v)
                    atomicAdd(&s_cnt[k], v);
            }
            __syncthreads();
            if (tid >= 1 && tid <= klds && s_cnt[tid])
                g_add(&acc->cnt[tid], (unsigned long long)s_cnt[tid]);
            if (tid >= 2 && tid <= klds + 1 && s_first[tid] != kNone)
                g_min(&acc->first[tid], s_first[tid]);
        }
        __syncthreads();
    };

    // phase clock (the PH instance only, for measurement): workgroup time per
    // phase of the segment loop from the constant-rate counter, summed in LDS
    // and added to L.phase once per workgroup at exit
    uint64_t t_ph = 0;
    if (PH && tid < 3)
        s_ph[tid] = 0;
    auto phase_tick = [&](int ph) {
        if (PH) {
            const uint64_t t = __builtin_amdgcn_s_memrealtime();
            if (ph >= 0 && tid == 0)
                atomicAdd(&s_ph[ph], (unsigned long long)(t - t_ph));
            t_ph = t;
        }
    };

    // optional start delay by launch-order slot (the workgroups sharing a CU
    // come from different quarters of the grid), so that their phases --
    // L2-bound init, LDS-bound marking, VALU-bound search -- do not line up
    if (L.stagger) {
        const uint32_t slot = (uint32_t)(((uint64_t)blockIdx.x * 4u) / gridDim.x);
        for (uint32_t i = 0; i < slot * L.stagger; i++)
            __builtin_amdgcn_s_sleep(1);
    }

    for (;;) {
        if (tid == 0) {
            uint32_t ok = 0, ivi = 0, b = 0, cnt = 0;
            if (L.items) {
                const uint32_t it = atomicAdd(L.queue, 1u);
                if (it < L.n_items) {
                    const uint4 x = L.items[it];
                    ok = 1;
                    ivi = x.x;
                    b = x.y;
                    cnt = x.z;
                }
            } else {
                // one interval: run `it` of L.n_items equal runs
                const uint32_t it = atomicAdd(L.queue, 1u);
                if (it < L.n_items) {
                    const uint64_t ns = L.iv[0].nseg;
                    ok = 1;
                    b = (uint32_t)((uint64_t)it * ns / L.n_items);
                    cnt = (uint32_t)((uint64_t)(it + 1) * ns / L.n_items) - b;
                }
            }
            s_item[0] = ivi;
            s_item[1] = b;
            s_item[2] = cnt;
            s_item[3] = ok;
        }
        __syncthreads();
        const uint32_t item_ok = rfl(s_item[3]);
        const uint32_t ivi = rfl(s_item[0]), seg0 = rfl(s_item[1]), nsegs = rfl(s_item[2]);
        // the partial totals of cur_iv go to its accumulators when the next
        // run belongs to another interval, when they would exceed kFlushSegs
        // segments (32-bit counters), and at exit: one round of global
        // atomics per flush instead of one per run
        if (cur_iv != ~0u && (!item_ok || ivi != cur_iv || acc_segs + nsegs > kFlushSegs)) {
            flush(cur_iv);
            cur_iv = ~0u;
        }
        if (!item_ok) {
            if (PH && tid < 3)
                atomicAdd(&L.phase[tid], s_ph[tid]);
            break;
        }
        if (cur_iv == ~0u) {
            if (tid < kMaxKh + 2)
                s_first[tid] = kNone;
            if (tid <= kMaxKh)
                s_cnt[tid] = 0;
#pragma unroll
            for (int k = 0; k <= kRegLevels; k++)
                cnt[k] = 0;
            found = 0;
            acc_segs = 0;
            cur_iv = ivi;
            __syncthreads();
        }
        acc_segs += nsegs;
        const Interval IV = L.iv[ivi];
        const uint32_t cap = L.bucket_cap;
        // The issue arbiter favours older waves, so of the workgroups sharing
        // a CU the first-launched would finish far ahead of the last.  Raising
        // the priority of a workgroup with more of its run left keeps them
        // level, and the CU busy until the end.
        // Step 1 of a segment: the words of the two tables (9, 25, 49 and
        // 121, 169) ORed into the region whose first word is gw0 (table 1 at
        // offset wb), by the nl lanes lid < nl, from pair `first` on (the
        // caller wrote the pairs below first * nl); words below odd index 0
        // are all marked.  16-byte loads (two words per lane; the tables need
        // only 8-byte alignment for global loads), 16-byte LDS stores; byte
        // offsets are 32-bit so that a load is a scalar base plus one lane
        // offset.
        auto init_region = [&](int64_t gw0, uint32_t wb, uint32_t lid, uint32_t nl, uint32_t first) {
            int64_t g2 = gw0 % (int64_t)kWheel2Period;
            if (g2 < 0)
                g2 += kWheel2Period;
            const char* src = reinterpret_cast<const char*>(L.wheel + wb);
            const char* src2 = reinterpret_cast<const char*>(L.wheel2 + g2);
            char* dst = reinterpret_cast<char*>(bm);
            if (gw0 >= 0) {
                const uint32_t st = 16 * nl;
                const uint32_t pairs = L.rw / 2;
                constexpr int kInitPairs = 2;  // pairs per lane in flight (VGPR budget)
                const uint32_t passes = (pairs - first * nl) / (kInitPairs * nl);
                uint32_t off = 16 * lid + first * st;
                for (uint32_t ps = 0; ps < passes; ps++, off += kInitPairs * st) {
                    u64x2 v[kInitPairs], x[kInitPairs];
                    uint32_t o[kInitPairs];
#pragma unroll
                    for (int u = 0; u < kInitPairs; u++) {
                        // each pair's offset as its own 32-bit value, so that
                        // its loads keep the scalar-base form
                        o[u] = off + u * st;
                        if (u > 0)
                            asm volatile("" : "+v"(o[u]));
                        v[u] = *reinterpret_cast<const u64x2*>(src + o[u]);
                        x[u] = *reinterpret_cast<const u64x2*>(src2 + o[u]);
                    }
#pragma unroll
                    for (int u = 0; u < kInitPairs; u++)
                        *reinterpret_cast<u64x2*>(dst + o[u]) = v[u] | x[u];
                }
                for (; off < 16 * pairs; off += st)
                    *reinterpret_cast<u64x2*>(dst + off) =
                        *reinterpret_cast<const u64x2*>(src + off) |
                        *reinterpret_cast<const u64x2*>(src2 + off);
                if ((L.rw & 1u) && lid == 0) {
                    const uint32_t o = 8 * (L.rw - 1);
                    *reinterpret_cast<uint64_t*>(dst + o) =
                        *reinterpret_cast<const uint64_t*>(src + o) |
                        *reinterpret_cast<const uint64_t*>(src2 + o);
                }
                // at origin 1 a region whose first word starts at odd index 0
                // has bit 0 at odd index -1, not positive: marked (lane 0
                // wrote word 0 itself)
                if (gw0 == 0 && L.origin && lid == 0)
                    bm[0] |= 1ull;
            } else {
                // words below odd index 0 are all marked; at origin 1 the word
                // at index 0 starts with odd index -1, marked too
                for (uint32_t w = lid; w < L.rw; w += nl)
                    bm[w] = (gw0 + (int64_t)w < 0)
                                ? ~0ull
                                : (reinterpret_cast<const uint64_t*>(src)[w] |
                                   reinterpret_cast<const uint64_t*>(src2)[w] |
                                   (gw0 + (int64_t)w == 0 ? (uint64_t)L.origin : 0ull));
            }
        };
        // each medium prime's first hit in the region whose bit 0 is odd index
        // B1, by the nl lanes lid < nl: from scratch for a run's first segment,
        // else one segment on from the last
        auto first_hits = [&](int64_t B1, bool restart, uint32_t lid, uint32_t nl) {
            if (restart) {
                for (uint32_t i = lid; i < nmed; i += nl) {
                    const uint32_t q = s_medq[i].x;
                    const int64_t d = (int64_t)((q - 1) >> 1) - B1;
                    int64_t f = d % (int64_t)q;
                    if (f < 0)
                        f += q;
                    s_f[i] = (uint32_t)f;
                }
            } else {
                for (uint32_t i = lid; i < nmed; i += nl) {
                    const uint2 qs = s_medq[i];
                    const uint32_t f = s_f[i];
                    s_f[i] = f >= qs.y ? f - qs.y : f + qs.x - qs.y;
                }
            }
        };
        auto set_priority = [&](uint32_t seg) {
            if (L.priority) {
                const uint32_t q = min(((seg0 + nsegs - seg) * 4u) / nsegs, 3u);
                if (q == 0)
                    __builtin_amdgcn_s_setprio(0);
                else if (q == 1)
                    __builtin_amdgcn_s_setprio(1);
                else if (q == 2)
                    __builtin_amdgcn_s_setprio(2);
                else
                    __builtin_amdgcn_s_setprio(3);
            }
        };

        // Algorithm 1 alone, with the waves in two roles.  A wave's vector
        // loads and stores complete on one counter, so a wave that has stores
        // in flight and then needs a load's result waits for the stores too;
        // the compiler, not knowing which lanes take which branch, places
        // such waits on every path it cannot rule out.  So the storers (upper
        // half of the waves) run a loop of their own with no global load in
        // it: they take the medium primes' first hits, mark, and write the
        // bitmap out, and their stores drain while the loaders (lower half)
        // load the next segment's tables and hit slots.  Both loops meet at
        // the same three barriers per segment.  Needs the task table in LDS
        // and an even number of waves.
        const bool split = MODE == 2 && L.tasks_in_lds && T % 128 == 0;
        if (split) {
            const uint32_t TL = T / 2, TS = T - TL;
            // wave-uniform (TL is a multiple of 64), and known to be so: each
            // wave runs exactly one of the two loops
            const bool loader = rfl(tid) < TL;
            const uint64_t n_bits = IV.I1 - IV.I0;
            const uint32_t sh = IV.out_shift;
            auto mark_medium = [&]() {
                for (uint32_t e = tid; e < L.n_tasks; e += T) {
                    const uint2 tk = s_task[e];
                    const uint32_t idx = tk.x >> 21, step = tk.y;
                    for (uint32_t pos = s_f[idx] + (tk.x & 0x1fffffu); pos < R; pos += step)
                        mark(bm32, pos);
                }
            };
            if (loader) {
                constexpr int kPre = 4;  // pairs per lane fetched a segment ahead
                u64x2 pre_v[kPre], pre_x[kPre];
                bool have_pre = false;
                const uint32_t pairs = L.rw / 2;
                for (uint32_t seg = seg0; seg < seg0 + nsegs; seg++) {
                    phase_tick(-1);
                    set_priority(seg);
                    const int64_t Bs = IV.A0 - (int64_t)HW * 64 + (int64_t)seg * (int64_t)S;
                    const int64_t B1 = Bs - (int64_t)L.origin;
                    const int64_t gw0 = Bs / 64;
                    const uint32_t wb = (uint32_t)(((uint64_t)IV.wheel_base0 + (uint64_t)seg * wstep) % kWheelPeriod);
                    const uint32_t gs = IV.seg_base + seg;
                    // the hit-slot count and first slot, then the tables (as
                    // in the single-role loop, over the loader lanes)
                    uint32_t nb = 0, slot_pos = R;
                    if (L.bucket_cnt) {
                        nb = *(const __attribute__((address_space(4))) uint32_t*)(uintptr_t)(L.bucket_cnt + gs);
                        if (nb <= cap && tid < nb)
                            slot_pos = L.bucket_slot[(uint64_t)gs * cap + tid];
                    }
                    uint32_t first = 0;  // pairs per lane fetched a segment ahead
                    if (have_pre && gw0 >= 0) {
#pragma unroll
                        for (int u = 0; u < kPre; u++)
                            *reinterpret_cast<u64x2*>(reinterpret_cast<char*>(bm) + 16 * (tid + u * TL)) =
                                pre_v[u] | pre_x[u];
                        first = kPre;
                    }
                    init_region(gw0, wb, tid, TL, first);
                    __syncthreads();
                    phase_tick(0);

                    // medium primes (both roles), the hit slots (loaders)
                    mark_medium();
                    if (L.bucket_cnt) {
                        if (nb <= cap) {
                            if (slot_pos < R)
                                mark(bm32, slot_pos);
                            const uint32_t* sl = L.bucket_slot + (uint64_t)gs * cap;
                            for (uint32_t e = tid + TL; e < nb; e += TL) {
                                const uint32_t pos = sl[e];
                                if (pos < R)
                                    mark(bm32, pos);
                            }
                        } else {
                            for (uint32_t pi = L.med_end + tid; pi < IV.pmax_end; pi += TL) {
                                const uint64_t p = L.primes[pi];
                                const uint64_t q = p * p;
                                for (uint64_t pos = first_hit(B1, q); pos < R; pos += q)
                                    mark(bm32, (uint32_t)pos);
                            }
                        }
                    }
                    __syncthreads();
                    phase_tick(1);

                    // the next segment's first kPre pairs per lane, at the
                    // addresses its init uses
                    have_pre = seg + 1 < seg0 + nsegs && gw0 + (int64_t)SW >= 0 && pairs / TL >= (uint32_t)kPre;
                    if (have_pre) {
                        const int64_t gwn = gw0 + (int64_t)SW;
                        const uint32_t wbn = wb + wstep >= kWheelPeriod ? wb + wstep - kWheelPeriod : wb + wstep;
                        const char* sn = reinterpret_cast<const char*>(L.wheel + wbn);
                        const char* sn2 = reinterpret_cast<const char*>(L.wheel2 + gwn % (int64_t)kWheel2Period);
#pragma unroll
                        for (int u = 0; u < kPre; u++) {
                            uint32_t o = 16 * tid + u * 16 * TL;
                            if (u > 0)
                                asm volatile("" : "+v"(o));
                            pre_v[u] = *reinterpret_cast<const u64x2*>(sn + o);
                            pre_x[u] = *reinterpret_cast<const u64x2*>(sn2 + o);
                        }
                    }
                    __syncthreads();
                    phase_tick(2);
                }
            } else {
                const uint32_t sid = tid - TL;
                for (uint32_t seg = seg0; seg < seg0 + nsegs; seg++) {
                    phase_tick(-1);
                    set_priority(seg);
                    const int64_t B1 = IV.A0 - (int64_t)HW * 64 + (int64_t)seg * (int64_t)S - (int64_t)L.origin;
                    first_hits(B1, seg == seg0, sid, TS);
                    __syncthreads();
                    phase_tick(0);

                    mark_medium();
                    __syncthreads();
                    phase_tick(1);

                    // the segment's output words (as in the single-role loop)
                    const uint64_t wo0 = (uint64_t)seg * SW;
                    if (wo0 * 64 + (uint64_t)SW * 64 <= n_bits && (((uintptr_t)IV.out_bits) & 15u) == 0) {
                        for (uint32_t lw = 2 * sid; lw < SW; lw += 2 * TS) {
                            const uint64_t w0 = bm[lw], w1 = bm[lw + 1], w2 = bm[lw + 2];
                            u64x2 o;
                            o.x = ~(sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0);
                            o.y = ~(sh ? ((w1 >> sh) | (w2 << (64 - sh))) : w1);
                            *(g_u64x2*)((g_u64*)IV.out_bits + wo0 + lw) = o;
                        }
                    } else {
                        for (uint32_t lw = sid; lw < SW; lw += TS) {
                            const uint64_t wo = wo0 + lw;
                            if (wo * 64 >= n_bits)
                                break;
                            const uint64_t lo = bm[lw], hi = bm[lw + 1];
                            uint64_t out = ~(sh ? ((lo >> sh) | (hi << (64 - sh))) : lo);
                            const uint64_t rem = n_bits - wo * 64;
                            if (rem < 64)
                                out &= (1ull << rem) - 1;
                            ((g_u64*)IV.out_bits)[wo] = out;
                        }
                    }
                    __syncthreads();
                    phase_tick(2);
                }
            }
        }

        for (uint32_t seg = seg0; seg < seg0 + nsegs && !split; seg++) {
            phase_tick(-1);
            set_priority(seg);
            // the region's words start at odd index Bs (a multiple of 64) for
            // the wheel tables (at the launch's origin); its bit 0 is odd index
            // B1 = Bs - origin
            const int64_t Bs = IV.A0 - (int64_t)HW * 64 + (int64_t)seg * (int64_t)S;
            const int64_t B1 = Bs - (int64_t)L.origin;
            const int64_t gw0 = Bs / 64;  // exact: Bs is a multiple of 64
            const uint32_t wb = (uint32_t)(((uint64_t)IV.wheel_base0 + (uint64_t)seg * wstep) % kWheelPeriod);

            // 0. the segment's hit-slot count and this lane's first slot, fetched
            //    now so that their latency overlaps the wheel loads
            const uint32_t gs = IV.seg_base + seg;
            uint32_t nb = 0, slot_pos = R;
            if (L.bucket_cnt) {
                // read-only here: a scalar (constant address space) load
                nb = *(const __attribute__((address_space(4))) uint32_t*)(uintptr_t)(L.bucket_cnt + gs);
                if (nb <= cap && tid < nb)
                    slot_pos = L.bucket_slot[(uint64_t)gs * cap + tid];
            }

            // 1. the wheel: odd multiples of 9, 25, 49 and of 121, 169 from the
            //    two tables; each medium prime's first hit in the region
            init_region(gw0, wb, tid, T, 0);
            first_hits(B1, seg == seg0, tid, T);
            __syncthreads();
            phase_tick(0);

            // 2. odd multiples of p^2: medium primes by lane-tasks, larger ones
            //    from the segment's hit slots (directly if the slots overflowed)
            // A prime with h = ceil(R / q) hits per region has c <= h tasks, so
            // c q <= R + q and f + v q < R + q: 32-bit positions suffice.
            // a task carries its start past the prime's first hit (v q, 21
            // bits), the prime's index (11 bits) and its step c q: one LDS read
            // of the prime's offset, no multiply
            auto mark_tasks = [&](const uint2* tk_table) {
                for (uint32_t e = tid; e < L.n_tasks; e += T) {
                    const uint2 tk = tk_table[e];
                    const uint32_t idx = tk.x >> 21, step = tk.y;
                    for (uint32_t pos = s_f[idx] + (tk.x & 0x1fffffu); pos < R; pos += step)
                        mark(bm32, pos);
                }
            };
            if (L.tasks_in_lds)
                mark_tasks(s_task);
            else
                mark_tasks(L.tasks);
            if (L.bucket_cnt) {
                if (nb <= cap) {
                    if (slot_pos < R)
                        mark(bm32, slot_pos);
                    const uint32_t* sl = L.bucket_slot + (uint64_t)gs * cap;
                    for (uint32_t e = tid + T; e < nb; e += T) {
                        const uint32_t pos = sl[e];
                        if (pos < R)
                            mark(bm32, pos);
                    }
                } else {
                    // slots overflowed: every prime above the medium range, directly
                    for (uint32_t pi = L.med_end + tid; pi < IV.pmax_end; pi += T) {
                        const uint64_t p = L.primes[pi];
                        const uint64_t q = p * p;
                        for (uint64_t pos = first_hit(B1, q); pos < R; pos += q)
                            mark(bm32, (uint32_t)pos);
                    }
                }
            }
            __syncthreads();
            phase_tick(1);

            if (MODE == 2) {
                // output word wo = seg * SW + lw covers odd indices I0 + 64 wo ...:
                // region bits out_shift + 64 lw ... (words lw and lw + 1)
                const uint32_t sh = IV.out_shift;
                const uint64_t n_bits = IV.I1 - IV.I0;
                const uint64_t wo0 = (uint64_t)seg * SW;
                auto store_pair = [&](uint32_t lw) {
                    const uint64_t w0 = bm[lw], w1 = bm[lw + 1], w2 = bm[lw + 2];
                    u64x2 o;
                    o.x = ~(sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0);
                    o.y = ~(sh ? ((w1 >> sh) | (w2 << (64 - sh))) : w1);
                    *(g_u64x2*)((g_u64*)IV.out_bits + wo0 + lw) = o;
                };
                if (wo0 * 64 + (uint64_t)SW * 64 <= n_bits && (((uintptr_t)IV.out_bits) & 15u) == 0) {
                    // a whole segment of output: two words per lane, 16-byte stores
                    for (uint32_t lw = 2 * tid; lw < SW; lw += 2 * T)
                        store_pair(lw);
                } else {
                    for (uint32_t lw = tid; lw < SW; lw += T) {
                        const uint64_t wo = wo0 + lw;
                        if (wo * 64 >= n_bits)
                            break;
                        const uint64_t lo = bm[lw], hi = bm[lw + 1];
                        const uint64_t v = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
                        uint64_t out = ~v;
                        const uint64_t rem = n_bits - wo * 64;
                        if (rem < 64)
                            out &= (1ull << rem) - 1;
                        ((g_u64*)IV.out_bits)[wo] = out;
                    }
                }
                __syncthreads();
                phase_tick(2);
                continue;
            }

            // 3. Algorithm 2, bit-sliced: (uhi:ulo) holds the n of one word
            //    still without a representation; step k keeps the n whose
            //    n - 2^k (2^(k-1) bits lower) is marked.  cnt[k] counts them
            //    after step k; s_first[k+1] collects the least such n.
            const uint64_t As = (uint64_t)(IV.A0 + (int64_t)seg * (int64_t)S);
            // main words wholly inside [I0, I1)
            uint32_t lo_w = 0, hi_w = SW;
            if (IV.I0 > As)
                lo_w = (uint32_t)min((IV.I0 - As + 63) / 64, (uint64_t)SW);
            if (IV.I1 < As + S)
                hi_w = IV.I1 > As ? (uint32_t)((IV.I1 - As) / 64) : 0u;
            // A segment whose main words all lie inside [I0, I1) and split
            // evenly over the workgroup, searched to the deepest in-LDS level,
            // takes the fast form: every lane active, every n valid, no
            // per-word index arithmetic, no level bound.
            const bool fast = lo_w == 0 && hi_w == SW && SW % T == 0 && klds == (uint32_t)kMaxKh;
            // per-n mode, FAST segments: a wave's 64 words are 4096 consecutive
            // output bytes, staged through LDS; every run of the segment starts
            // the same delta bytes past a 16-byte boundary
            const bool stage_ok = MODE == 1 && L.stage && IV.out_mink;
            const uint32_t delta = rfl((uint32_t)(((uintptr_t)IV.out_mink + (uintptr_t)(As - IV.I0)) & 15u));
            const uint32_t iters = (SW + T - 1) / T;
            // STEADY: the least n of depth 2 .. 5 have been offered already, so
            // steps 1 .. 4 run without any branch.
            const uint64_t* pbase = bm + HW + tid - 1;  // FAST: word before pass 0's word
            auto word_pass = [&](auto fast_c, auto steady_c, uint32_t itw) {
                constexpr bool FAST = decltype(fast_c)::value;
                constexpr bool STEADY = decltype(steady_c)::value;
                // the word's first n-index, for the rare paths only (formed from
                // an opaque copy of tid, so that no index arithmetic is hoisted
                // into the common path)
                auto j0_of = [&]() {
                    uint32_t t = tid;
                    asm volatile("" : "+v"(t));
                    return As + (uint64_t)(t + itw * T) * 64;
                };
                const uint32_t mw = tid + itw * T;
                const bool act = FAST || mw < SW;
                // pw points at the word before this lane's word (FAST: from the
                // loop-invariant base, one add per pass)
                const uint64_t* pw = FAST ? pbase + itw * T : bm + HW + (act ? mw : 0u) - 1;
                uint64_t V;
                if (FAST)
                    V = ~0ull;
                else if (!act)
                    V = 0;
                else if (mw >= lo_w && mw < hi_w)
                    V = ~0ull;
                else
                    V = valid_mask(As + (uint64_t)mw * 64, IV.I0, IV.I1);
                const uint64_t cur = pw[1], prv = pw[0];
                const uint32_t clo = (uint32_t)cur, chi = (uint32_t)(cur >> 32);
                const uint32_t plo = (uint32_t)prv, phi = (uint32_t)(prv >> 32);
                uint32_t ulo = (uint32_t)V, uhi = (uint32_t)(V >> 32);
                // per-n depths as bit planes: the step sets U_0 = V, U_1, U_2, ...
                // are nested, so the least k of an n, the number of sets that
                // hold it, has bit b equal to the parity of its membership in
                // the U_j with j = 2^b - 1 (mod 2^b)
                uint32_t pl[4][2] = {{(uint32_t)V, (uint32_t)(V >> 32)}, {0u, 0u}, {0u, 0u}, {0u, 0u}};
                found = rfl(found);
                bool alive = true;  // wave-uniform: some lane still has an n left
#pragma unroll
                for (int k = 1; k <= kMaxKh; k++) {
                    if (!FAST && k > (int)klds)
                        break;
                    // The region's bit 0 is one odd index below its first word
                    // boundary, so bit b of a word holds the odd index one below
                    // the word's n-bit b: n - 2^k, 2^(k-1) positions below n, is
                    // t = 2^(k-1) - 1 bits below in the bitmap.  k = 1 reads the
                    // word itself; k <= 7 funnel-shifts it with the word below
                    // by t; from k = 8 on the two words d = 2^(k-7) and d - 1
                    // below, shifted by 63.
                    uint32_t wlo, whi;
                    if (k == 1) {
                        wlo = clo;
                        whi = chi;
                    } else if (k <= 6) {
                        const uint32_t sh = 33u - (1u << (k - 1));
                        wlo = __builtin_amdgcn_alignbit(clo, phi, sh);
                        whi = __builtin_amdgcn_alignbit(chi, clo, sh);
                    } else if (k == 7) {
                        wlo = __builtin_amdgcn_alignbit(phi, plo, 1);
                        whi = __builtin_amdgcn_alignbit(clo, phi, 1);
                    } else {
                        const bool any = (ulo | uhi) != 0;
                        const uint64_t y = any ? pw[1 - (1 << (k - 7))] : 0ull;
                        const uint64_t x = any ? pw[2 - (1 << (k - 7))] : 0ull;
                        wlo = __builtin_amdgcn_alignbit((uint32_t)(y >> 32), (uint32_t)y, 1);
                        whi = __builtin_amdgcn_alignbit((uint32_t)x, (uint32_t)(y >> 32), 1);
                    }
                    ulo &= wlo;
                    uhi &= whi;
                    // levels below 4 are counted here; from level 4 on, where
                    // the empty-wave test runs first, after that test (a wave
                    // that stops there has nothing to count)
                    if (k < 4)
                        cnt[k] = bcnt_acc(uhi, bcnt_acc(ulo, cnt[k]));
                    if (MODE == 1) {
#pragma unroll
                        for (int b = 0; b < 4; b++) {
                            if ((k & ((1 << b) - 1)) == (1 << b) - 1) {
                                pl[b][0] ^= ulo;
                                pl[b][1] ^= uhi;
                            }
                        }
                    }
                    // a wave of 4096 n almost never empties before step 4, so
                    // the test for an empty wave starts there
                    const bool track = !(STEADY && k <= 4) && !(found & (1u << (k + 1)));
                    if (k >= 4 || track) {
                        const uint64_t bal = __ballot((ulo | uhi) != 0);
                        if (bal == 0) {
                            alive = false;
                            break;
                        }
                        if (k >= 4) {
                            if (k <= kRegLevels)
                                cnt[k] = bcnt_acc(uhi, bcnt_acc(ulo, cnt[k]));
                            else if (ulo | uhi)
                                atomicAdd(&s_cnt[k], (uint32_t)(__popc(ulo) + __popc(uhi)));
                        }
                        if (track) {
                            const uint32_t l = rfl((uint32_t)(__ffsll((unsigned long long)bal) - 1));
                            if (lane == l) {
                                const uint64_t U = ((uint64_t)uhi << 32) | ulo;
                                const uint64_t n_first = j0_of() +
                                                         (uint64_t)(__ffsll((unsigned long long)U) - 1);
                                atomicMin(&s_first[k + 1], (unsigned long long)n_first);
                            }
                            found |= 1u << (k + 1);
                        }
                    }
                }
                // the loop ends early (alive false) for all but the rarest words
                const uint64_t U = ((uint64_t)uhi << 32) | ulo;
                // still unresolved after the in-LDS steps: to the exact tail
                // pass -- unless the search limit is the in-LDS depth, so that
                // these n are exceptions already counted in cnt[k_lds]; then
                // they are listed only when the call lists exceptions
                const bool no_tail = klds >= L.kmax_eff;
                if (__builtin_expect(alive, 0) && U && (!no_tail || L.exc_list)) {
                    // one reservation of popcount(U) list entries per word
                    const uint64_t j0 = j0_of();
                    const unsigned long long c = (unsigned long long)__popcll(U);
                    g_add(&IV.acc->tail_count, c);
                    unsigned long long idx = atomicAdd(L.tail_count, c);
                    for (uint64_t x = U; x; idx++) {
                        const int bit = __ffsll((unsigned long long)x) - 1;
                        x &= x - 1;
                        if (idx < L.tail_cap) {
                            L.tail_n[idx] = j0 + (uint64_t)bit;
                            L.tail_iv[idx] = ivi;
                        } else {
                            g_or(&IV.acc->status, no_tail ? (unsigned)ESQ_STATUS_EXCEPTIONS_INCOMPLETE
                                                              : (unsigned)ESQ_STATUS_TAIL_OVERFLOW);
                        }
                    }
                }
                if (MODE == 1 && IV.out_mink) {
                    // n without a representation yet (the tail pass decides
                    // them) get 0
#pragma unroll
                    for (int b = 0; b < 4; b++) {
                        pl[b][0] &= ~ulo;
                        pl[b][1] &= ~uhi;
                    }
                    // planes -> one byte per n: nibble t of plane b spread to
                    // bit b of 4 bytes.  Plane 2 (least k in 4 .. 7) holds
                    // 1.4e-4 of the n, so a wave of 4096 n has none more often
                    // than not, and plane 3 (k >= 8) is almost never set: both
                    // are spread only when some lane of the wave has a bit
                    uint32_t D[16];
#pragma unroll
                    for (int t = 0; t < 16; t++) {
                        const int h = t >> 3, sh = 4 * (t & 7);
                        D[t] = (((pl[0][h] >> sh) & 15u) * 0x00204081u & 0x01010101u) |
                               (((pl[1][h] >> sh) & 15u) * 0x00408102u & 0x02020202u);
                    }
                    if (__ballot((pl[2][0] | pl[2][1]) != 0)) {
#pragma unroll
                        for (int t = 0; t < 16; t++)
                            D[t] |= spread4((pl[2][t >> 3] >> (4 * (t & 7))) & 15u) << 2;
                    }
                    if (__ballot((pl[3][0] | pl[3][1]) != 0)) {
#pragma unroll
                        for (int t = 0; t < 16; t++)
                            D[t] |= spread4((pl[3][t >> 3] >> (4 * (t & 7))) & 15u) << 3;
                    }
                    if (FAST && stage_ok) {
                        g_u8* o = (g_u8*)IV.out_mink + (As - IV.I0) + (uint64_t)(itw * T + (tid & ~63u)) * 64;
                        switch ((delta + 3) >> 2) {
                        case 0: stage_store_run<0>(s_stage, o, D, lane, delta); break;
                        case 1: stage_store_run<1>(s_stage, o, D, lane, delta); break;
                        case 2: stage_store_run<2>(s_stage, o, D, lane, delta); break;
                        case 3: stage_store_run<3>(s_stage, o, D, lane, delta); break;
                        default: stage_store_run<4>(s_stage, o, D, lane, delta); break;
                        }
                    } else if (V) {
                        const uint64_t j0 = As + (uint64_t)mw * 64;
                        store_depths((g_u8*)IV.out_mink + ((int64_t)j0 - (int64_t)IV.I0), D, V);
                    }
                }
            };
            constexpr uint32_t kSteadyBits = 0x3Cu;  // levels 2 .. 5
            uint32_t itw = 0;
            if (fast) {
                for (; itw < iters && (rfl(found) & kSteadyBits) != kSteadyBits; itw++)
                    word_pass(std::true_type{}, std::false_type{}, itw);
                for (; itw < iters; itw++)
                    word_pass(std::true_type{}, std::true_type{}, itw);
            } else {
                for (; itw < iters; itw++)
                    word_pass(std::false_type{}, std::false_type{}, itw);
            }
            __syncthreads();
            phase_tick(2);
        }

        // the item's s_item slots are reused by the next fetch
        __syncthreads();
    }
}

size_t verify_lds_bytes(const Launch& L, uint32_t block)
{
    return verify_lds_size(L.rw, L.med_end - kFirstMedium, L.tasks_in_lds ? L.n_tasks : 0u, L.stage != 0,
                           block);
}

hipError_t launch_verify(const Launch& L, uint32_t grid, uint32_t block, hipStream_t s)
{
    const size_t lds = verify_lds_bytes(L, block);
    if (grid == 0 || L.n_items == 0)
        return hipSuccess;
    // the phase-clock instances only when the clock is on
    switch (L.mode * 2 + (L.phase ? 1 : 0)) {
    case 0:
        hipLaunchKernelGGL((k_verify<0, false>), dim3(grid), dim3(block), lds, s, L);
        break;
    case 1:
        hipLaunchKernelGGL((k_verify<0, true>), dim3(grid), dim3(block), lds, s, L);
        break;
    case 2:
        hipLaunchKernelGGL((k_verify<1, false>), dim3(grid), dim3(block), lds, s, L);
        break;
    case 3:
        hipLaunchKernelGGL((k_verify<1, true>), dim3(grid), dim3(block), lds, s, L);
        break;
    case 4:
        hipLaunchKernelGGL((k_verify<2, false>), dim3(grid), dim3(block), lds, s, L);
        break;
    default:
        hipLaunchKernelGGL((k_verify<2, true>), dim3(grid), dim3(block), lds, s, L);
        break;
    }
    return hipGetLastError();
}

int verify_occupancy(int mode, uint32_t block, size_t lds_bytes)
{
    int occ = 0;
    hipError_t e;
    if (mode == 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_verify<1>, (int)block, lds_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_verify<0>, (int)block, lds_bytes);
    if (e != hipSuccess)
        return 1;
    return occ > 0 ? occ : 1;
}


// --------------------------------------------------------------- tail

// Exact search, by trial division over the resident prime squares, for the
// n whose first k_lds candidates were all marked (Algorithm 2 continued).
__global__ __launch_bounds__(256) void k_tail(Launch L)
{
    __shared__ int s_hit;
    const unsigned long long total = *L.tail_count;
    const uint64_t count = total < L.tail_cap ? total : L.tail_cap;
    volatile int* hitp = &s_hit;
    for (uint64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const uint64_t j = L.tail_n[idx];
        if (L.k_lds >= L.kmax_eff) {
            // listed exceptions: no k is left to try, and the counts, first-n
            // slots and per-n bytes are complete already
            if (threadIdx.x == 0)
                L.tail_d[idx] = 0;
            continue;
        }
        const Interval IV = L.iv[L.tail_iv[idx]];
        const uint64_t n = 2 * j + 1;
        uint32_t d = 0;
        for (uint32_t k = L.k_lds + 1; k <= 63; k++) {
            if (k > L.kmax_eff)
                break;
            const uint64_t pk = 1ull << k;
            if (pk >= n)
                break;
            const uint64_t m = n - pk;
            if (threadIdx.x == 0)
                *hitp = 0;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < L.nprimes; i += blockDim.x) {
                const uint64_t pr = L.primes[i];
                const uint64_t q = pr * pr;
                if (q > m || *hitp)
                    break;
                if (m % q == 0) {
                    *hitp = 1;
                    break;
                }
            }
            __syncthreads();
            const int hit = *hitp;
            __syncthreads();
            if (!hit) {
                d = k;
                break;
            }
        }
        if (threadIdx.x == 0) {
            L.tail_d[idx] = (uint8_t)d;
            g_add(&IV.acc->deep_hist[d], 1ull);
            const uint32_t top = d ? d : 64u;
            for (uint32_t kk = L.k_lds + 2; kk <= top; kk++)
                g_min(&IV.acc->first[kk], (unsigned long long)j);
            if (IV.out_mink)
                ((g_u8*)IV.out_mink)[j - IV.I0] = (uint8_t)d;
        }
    }
}

hipError_t launch_tail(const Launch& L, hipStream_t s)
{
    hipLaunchKernelGGL(k_tail, dim3(512), dim3(256), 0, s, L);
    return hipGetLastError();
}

// ------------------------------------------------------------ finalize

__device__ unsigned long long block_sum(unsigned long long v, unsigned long long* s_acc)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    if (threadIdx.x == 0)
        *s_acc = 0;
    __syncthreads();
    if ((threadIdx.x & 63u) == 0)
        atomicAdd(s_acc, v);
    __syncthreads();
    const unsigned long long r = *s_acc;
    __syncthreads();
    return r;
}

// One workgroup per interval.
__global__ __launch_bounds__(1024) void k_finalize(Launch L, void* out_summaries, void* out_records,
                                                   uint64_t* out_exceptions, uint64_t exc_cap)
{
    extern __shared__ unsigned long long s_sort[];
    __shared__ unsigned long long s_acc;
    __shared__ unsigned int s_fill;
    __shared__ unsigned long long s_first[65];
    const uint32_t ivi = blockIdx.x;
    const Interval IV = L.iv[ivi];
    const Acc* A = IV.acc;
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const unsigned long long tail_total = *L.tail_count;
    const uint64_t nlist = tail_total < L.tail_cap ? tail_total : L.tail_cap;
    const uint64_t n_odd = IV.I1 - IV.I0;
    // with the search limit at the in-LDS depth there is no tail pass: the n
    // still unresolved after step k_lds are the exceptions, and they are
    // deeper than every level, so first[k] for k > k_lds + 1 is first[k_lds + 1]
    const bool no_tail = L.k_lds >= L.kmax_eff;
    const uint64_t n_exc = no_tail ? A->cnt[L.k_lds] : A->deep_hist[0];
    const uint64_t want = n_exc < exc_cap ? n_exc : exc_cap;
    for (uint32_t i = tid; i < 65; i += T)
        s_first[i] = (no_tail && i > L.k_lds + 1) ? A->first[L.k_lds + 1] : A->first[i];

    if (out_exceptions && want > 0) {
        // the want-th smallest exception of this interval (binary search on
        // its odd index), then an LDS sort of those up to it
        uint64_t thr = kNone;
        if (want < n_exc) {
            uint64_t lo = 0, hi = 1ull << 56;
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                unsigned long long c = 0;
                for (uint64_t i = tid; i < nlist; i += T)
                    c += (L.tail_iv[i] == ivi && L.tail_d[i] == 0 && L.tail_n[i] <= mid) ? 1ull : 0ull;
                c = block_sum(c, &s_acc);
                if (c >= want)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            thr = lo;
        }
        if (tid == 0)
            s_fill = 0;
        __syncthreads();
        for (uint64_t i = tid; i < nlist; i += T)
            if (L.tail_iv[i] == ivi && L.tail_d[i] == 0 && L.tail_n[i] <= thr) {
                const unsigned int slot = atomicAdd(&s_fill, 1u);
                if (slot < kFinalizeSortCap)
                    s_sort[slot] = L.tail_n[i];
            }
        __syncthreads();
        const uint32_t got = min(s_fill, kFinalizeSortCap);
        uint32_t n2 = 1;
        while (n2 < got)
            n2 <<= 1;
        for (uint32_t i = got + tid; i < n2; i += T)
            s_sort[i] = kNone;
        __syncthreads();
        for (uint32_t k = 2; k <= n2; k <<= 1)
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < n2; i += T) {
                    const uint32_t ixj = i ^ j;
                    if (ixj > i) {
                        const unsigned long long a = s_sort[i], b = s_sort[ixj];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            s_sort[i] = b;
                            s_sort[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        for (uint32_t i = tid; i < want && i < got; i += T)
            out_exceptions[i] = 2 * s_sort[i] + 1;
    }
    __syncthreads();

    __shared__ unsigned long long h[65];
    __shared__ unsigned long long s_cnt[16];
    for (uint32_t i = tid; i < 65; i += T)
        h[i] = no_tail ? (i == 0 ? n_exc : 0ull) : A->deep_hist[i];
    for (uint32_t i = tid; i < 16; i += T)
        s_cnt[i] = A->cnt[i];
    __syncthreads();
    if (tid != 0)
        return;
    esq_summary* out = reinterpret_cast<esq_summary*>(out_summaries) + ivi;
    unsigned long long prev = n_odd;
    for (uint32_t k = 1; k <= L.k_lds; k++) {
        const unsigned long long c = s_cnt[k];
        h[k] = prev - c;   // the tail pass only fills depths above k_lds
        prev = c;
    }
    unsigned long long ksum = 0;
    uint32_t kseen = 0;
    for (uint32_t k = 1; k < 65; k++) {
        ksum += (unsigned long long)k * h[k];
        if (h[k])
            kseen = k;
    }
    // record-setters: first[k] = least n-index with depth >= k; each distinct
    // value is a record, labelled with the deepest level sharing it
    esq_record* rec = out_records ? reinterpret_cast<esq_record*>(out_records) + (uint64_t)ivi * ESQ_RECORDS_CAP
                                  : nullptr;
    uint32_t nrec = 0;
    if (n_odd) {
        uint32_t k = 1;
        while (k <= 64) {
            const unsigned long long v = (k == 1) ? IV.I0 : s_first[k];
            if (v == kNone)
                break;
            uint32_t kk = k;
            while (kk < 64 && s_first[kk + 1] == v)
                kk++;
            if (rec && nrec < ESQ_RECORDS_CAP) {
                const uint64_t n = 2 * v + 1;
                rec[nrec].n = n;
                rec[nrec].k = kk == 64 ? 0u : kk;
                // an exception found by the search limit, with a larger k
                // still positive, vs one for which every k with 2^k < n failed
                rec[nrec].flags = (kk == 64 && L.kmax_eff < 63 && (1ull << (L.kmax_eff + 1)) < n)
                                      ? (uint32_t)ESQ_RECORD_KMAX_LIMIT : 0u;
            }
            nrec++;
            k = kk + 1;
        }
    }
    out->n0 = n_odd ? 2 * IV.I0 + 1 : 0;
    out->n_odd = n_odd;
    for (int k = 0; k < 65; k++)
        out->hist[k] = h[k];
    out->ksum = ksum;
    out->kmax_seen = kseen;
    out->n_records = nrec < ESQ_RECORDS_CAP ? nrec : ESQ_RECORDS_CAP;
    out->n_exceptions = h[0];
    out->status = A->status;
    out->reserved = 0;
}

hipError_t launch_finalize(const Launch& L, void* out_summaries, void* out_records,
                           uint64_t* out_exceptions, uint64_t exc_cap, hipStream_t s)
{
    if (L.n_iv == 0)
        return hipSuccess;
    const size_t lds = out_exceptions ? (size_t)kFinalizeSortCap * 8 : 0;
    hipLaunchKernelGGL(k_finalize, dim3(L.n_iv), dim3(out_exceptions ? 1024 : 64), lds, s, L,
                       out_summaries, out_records, out_exceptions, exc_cap);
    return hipGetLastError();
}

hipError_t configure_kernels()
{
    hipError_t e;
    const int lds_max = (int)kVerifyLdsMax;
    const void* fns[6] = {(const void*)k_verify<0, false>, (const void*)k_verify<0, true>,
                          (const void*)k_verify<1, false>, (const void*)k_verify<1, true>,
                          (const void*)k_verify<2, false>, (const void*)k_verify<2, true>};
    for (const void* f : fns) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
        if (e != hipSuccess) return e;
    }
    e = hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kFinalizeSortCap * 8));
    return e;
}

}  // namespace esq
