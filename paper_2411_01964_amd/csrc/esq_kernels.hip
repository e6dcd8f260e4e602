// HIP kernels for gfx950 (wave64).  Exact integer work only: no floating
// point and no matrix cores -- the sieve and the search are bit operations.
//
//   k_wheel_build  periodic pattern of odd multiples of 9, 25, 49, 121
//   k_prepare      zero the per-call accumulators
//   k_bucket       large primes (p^2 above the LDS region): scatter every odd
//                  multiple of p^2 into per-segment hit lists (count / fill)
//   k_scan         exclusive scan of the per-segment hit counts
//   k_segment      one workgroup per segment: Algorithm 1 in LDS, then
//                  Algorithm 2 as a bit-sliced scan over the LDS bitmap
//   k_tail         exact search for the rare n not resolved from LDS
//   k_finalize     aggregates, record-setters, sorted exceptions
#include "esq_internal.h"
#include "esq.h"

namespace esq {

// ------------------------------------------------------------ wheel table

// Word w holds bits for odd indices 64w .. 64w+63 (mod kWheelPeriod).  An odd
// index x is an odd multiple of q = p^2 iff x = (q - 1)/2 (mod q).
__global__ void k_wheel_build(uint64_t* wheel, uint32_t nwords)
{
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
         w += gridDim.x * blockDim.x) {
        const uint32_t base = (uint32_t)(((uint64_t)w * 64u) % kWheelPeriod);
        uint64_t word = 0;
        for (uint32_t b = 0; b < 64; b++) {
            const uint32_t x = base + b;
            if (x % 9u == 4u || x % 25u == 12u || x % 49u == 24u || x % 121u == 60u)
                word |= 1ull << b;
        }
        wheel[w] = word;
    }
}

hipError_t launch_wheel_build(uint64_t* wheel, hipStream_t s)
{
    hipLaunchKernelGGL(k_wheel_build, dim3(1024), dim3(256), 0, s, wheel,
                       kWheelPeriod + kWheelExtra);
    return hipGetLastError();
}

// --------------------------------------------------------------- prepare

__global__ void k_prepare(Acc* acc, uint32_t* counts, uint32_t* cursor, uint32_t nseg)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = t; i < 65; i += stride) {
        acc->cnt[i] = 0;
        acc->first[i] = kNone;
        acc->deep_hist[i] = 0;
    }
    if (t == 0) {
        acc->tail_count = 0;
        acc->status = 0;
        acc->bucket_total = 0;
    }
    if (counts)
        for (uint32_t i = t; i < nseg; i += stride) {
            counts[i] = 0;
            cursor[i] = 0;
        }
}

hipError_t launch_prepare(Acc* acc, uint32_t* counts, uint32_t* cursor, uint32_t nseg,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_prepare, dim3(64), dim3(256), 0, s, acc, counts, cursor, nseg);
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

template <bool FILL>
__device__ __forceinline__ void bucket_put(const BucketParams& p, uint32_t seg, uint32_t off)
{
    if (!FILL) {
        atomicAdd(&p.counts[seg], 1u);
    } else {
        const uint32_t pos = atomicAdd(&p.cursor[seg], 1u);
        const uint64_t idx = (uint64_t)p.offsets[seg] + pos;
        if (idx < p.capacity)
            p.entries[idx] = off;
        else
            atomicOr(&p.acc->status, (unsigned)ESQ_STATUS_BUCKET_OVERFLOW);
    }
}

// Segment s covers y in [s S, s S + S + overlap): a hit belongs to segment
// floor(y / S) and to every earlier segment whose region still reaches it.
template <bool FILL>
__device__ __forceinline__ void bucket_emit(const BucketParams& p, uint64_t y)
{
    uint64_t seg = y >> p.log2S;
    uint64_t off = y & ((1ull << p.log2S) - 1);
    const uint64_t R = (1ull << p.log2S) + p.overlap;
    while (off < R) {
        if (seg < p.nseg)
            bucket_put<FILL>(p, (uint32_t)seg, (uint32_t)off);
        if (seg == 0)
            break;
        seg--;
        off += 1ull << p.log2S;
    }
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_bucket(BucketParams p)
{
    if (blockIdx.x < p.n_heavy) {
        // a prime with many hits: the workgroup strides over them
        const uint64_t pr = p.primes[p.p_begin + blockIdx.x];
        const uint64_t q = pr * pr;
        const uint64_t f = first_hit(p.B0, q);
        if (f >= p.E)
            return;
        const uint64_t nh = (p.E - 1 - f) / q + 1;
        for (uint64_t t = threadIdx.x; t < nh; t += blockDim.x)
            bucket_emit<FILL>(p, f + t * q);
    } else {
        const uint64_t i = (uint64_t)(blockIdx.x - p.n_heavy) * blockDim.x + threadIdx.x;
        if (i >= p.n_light)
            return;
        const uint64_t pr = p.primes[p.p_begin + p.n_heavy + i];
        const uint64_t q = pr * pr;
        for (uint64_t y = first_hit(p.B0, q); y < p.E; y += q)
            bucket_emit<FILL>(p, y);
    }
}

hipError_t launch_bucket(const BucketParams& p, bool fill, hipStream_t s)
{
    const uint32_t blocks = p.n_heavy + (p.n_light + 255) / 256;
    if (blocks == 0)
        return hipSuccess;
    if (fill)
        hipLaunchKernelGGL(k_bucket<true>, dim3(blocks), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(k_bucket<false>, dim3(blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_scan(const uint32_t* counts, uint32_t* offsets,
                                               uint32_t nseg, Acc* acc, uint64_t capacity)
{
    __shared__ unsigned long long part[1024];
    const uint32_t T = blockDim.x, t = threadIdx.x;
    const uint32_t per = (nseg + T - 1) / T;
    const uint32_t b = min(t * per, nseg), e = min(b + per, nseg);
    unsigned long long sum = 0;
    for (uint32_t i = b; i < e; i++)
        sum += counts[i];
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < T; off <<= 1) {
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - sum;
    for (uint32_t i = b; i < e; i++) {
        offsets[i] = (uint32_t)run;
        run += counts[i];
    }
    if (t == T - 1) {
        const unsigned long long tot = part[T - 1];
        offsets[nseg] = (uint32_t)tot;
        acc->bucket_total = (unsigned)(tot > 0xffffffffull ? 0xffffffffull : tot);
        if (tot > capacity)
            atomicOr(&acc->status, (unsigned)ESQ_STATUS_BUCKET_OVERFLOW);
    }
}

hipError_t launch_scan(const uint32_t* counts, uint32_t* offsets, uint32_t nseg, Acc* acc,
                       uint64_t capacity, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, offsets, nseg, acc, capacity);
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
__device__ __forceinline__ void store_depths(uint8_t* out, const uint32_t (&D)[16], uint64_t V)
{
    const uint32_t mis = (uint32_t)((uintptr_t)out & 3u);
    uint8_t* al = out - mis;
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
            *reinterpret_cast<uint32_t*>(al + 4 * t) = val;
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

// MODE 0: verify, aggregates only; MODE 1: verify + per-n bytes;
// MODE 2: Algorithm 1 alone, bitmap to HBM.
template <int MODE>
__global__ __launch_bounds__(1024) void k_segment(SegParams P)
{
    extern __shared__ uint64_t bm[];
    __shared__ uint32_t s_f[kMaxMedium];
    __shared__ uint32_t s_q[kMaxMedium];
    __shared__ uint32_t s_cnt[kMaxKh + 2];
    __shared__ uint32_t s_first[kMaxKh + 2];

    const uint32_t tid = threadIdx.x, T = blockDim.x, seg = blockIdx.x;
    const uint32_t S = 1u << P.log2S;
    const int64_t Bs = P.A0 - (int64_t)P.hlo_words * 64 + (int64_t)seg * (int64_t)S;
    const int64_t gw0 = Bs / 64;  // exact: Bs is a multiple of 64
    const uint32_t wb =
        (uint32_t)(((uint64_t)P.wheel_base0 + (uint64_t)seg * P.wheel_step) % kWheelPeriod);

    // 1. initialise: wheel pattern; words below odd index 0 are all "marked"
    for (uint32_t w = tid; w < P.rw; w += T)
        bm[w] = (gw0 + (int64_t)w < 0) ? ~0ull : P.wheel[wb + w];
    // first hit of each medium prime inside the region
    for (uint32_t i = tid; i < P.nmed; i += T) {
        const uint32_t pr = P.primes[P.med_begin + i];
        const uint32_t q = pr * pr;
        const int64_t d = (int64_t)((q - 1) >> 1) - Bs;
        int64_t f = d % (int64_t)q;
        if (f < 0)
            f += q;
        s_f[i] = (uint32_t)f;
        s_q[i] = q;
    }
    if (tid < kMaxKh + 2) {
        s_cnt[tid] = 0;
        s_first[tid] = kNone32;
    }
    __syncthreads();

    // 2. mark odd multiples of p^2: medium primes by lane-tasks, large ones
    //    from this segment's hit list
    uint32_t* bm32 = reinterpret_cast<uint32_t*>(bm);
    const uint32_t R = P.rw * 64;
    for (uint32_t e = tid; e < P.n_med_entries; e += T) {
        const MedEntry me = P.med[e];
        const uint32_t q = s_q[me.idx];
        const uint32_t v = me.vc & 0xffffu, c = me.vc >> 16;
        const uint64_t p0 = (uint64_t)s_f[me.idx] + (uint64_t)v * q;
        if (p0 >= R)
            continue;
        const uint32_t step = c * q;
        for (uint32_t pos = (uint32_t)p0; pos < R; pos += step)
            atomicOr(&bm32[pos >> 5], 1u << (pos & 31));
    }
    if (P.bucket_off) {
        const uint32_t b0 = P.bucket_off[seg];
        const uint32_t b1 = (uint32_t)min((uint64_t)P.bucket_off[seg + 1], P.bucket_cap);
        for (uint32_t e = b0 + tid; e < b1; e += T) {
            const uint32_t pos = P.bucket_ent[e];
            if (pos < R)
                atomicOr(&bm32[pos >> 5], 1u << (pos & 31));
        }
    }
    __syncthreads();

    if (MODE == 2) {
        // output word wo = seg * S/64 + lw covers odd indices I0 + 64 wo ...:
        // region bits out_shift + 64 lw ... (words lw and lw + 1)
        const uint32_t SW = S / 64;
        const uint32_t sh = P.out_shift;
        for (uint32_t lw = tid; lw < SW; lw += T) {
            const uint64_t wo = (uint64_t)seg * SW + lw;
            if (wo * 64 >= P.n_bits)
                break;
            const uint64_t lo = bm[lw], hi = bm[lw + 1];
            const uint64_t v = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
            uint64_t out = ~v;
            const uint64_t rem = P.n_bits - wo * 64;
            if (rem < 64)
                out &= (1ull << rem) - 1;
            P.out_bits[wo] = out;
        }
        return;
    }

    // 3. Algorithm 2, bit-sliced: U holds the n of one word still without a
    //    representation; step k keeps n whose n - 2^k (2^(k-1) bits lower) is
    //    marked.  cnt[k] counts U after step k; s_first[k+1] the first n in it.
    const uint32_t HW = P.hlo_words;
    const uint64_t As = (uint64_t)(P.A0 + (int64_t)seg * (int64_t)S);
    const uint32_t lane = tid & 63u;
    const uint32_t klds = P.k_lds;
    uint32_t cnt[kMaxKh + 1];
#pragma unroll
    for (int k = 0; k <= kMaxKh; k++)
        cnt[k] = 0;
    uint32_t found = 0;

    for (uint32_t w = HW + tid; w < P.rw; w += T) {
        const uint64_t j0 = As + (uint64_t)(w - HW) * 64;
        const uint64_t V = valid_mask(j0, P.I0, P.I1);
        uint64_t U = V;
        const uint64_t cur = bm[w], prv = bm[w - 1];
        uint32_t D[16];
        if (MODE == 1) {
#pragma unroll
            for (int i = 0; i < 16; i++)
                D[i] = spread4((uint32_t)(V >> (4 * i)) & 15u);
        }
#pragma unroll
        for (int k = 1; k <= kMaxKh; k++) {
            if (k > (int)klds)
                break;
            uint64_t win;
            if (k <= 6) {
                const int sh = 1 << (k - 1);
                win = (cur << sh) | (prv >> (64 - sh));
            } else if (k == 7) {
                win = prv;
            } else {
                win = U ? bm[w - (1u << (k - 7))] : 0ull;
            }
            U &= win;
            cnt[k] += (uint32_t)__popcll(U);
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < 16; i++)
                    D[i] += spread4((uint32_t)(U >> (4 * i)) & 15u);
            }
            const uint64_t b = __ballot(U != 0);
            if (b == 0)
                break;
            if (!(found & (1u << (k + 1)))) {
                const int l = __ffsll((unsigned long long)b) - 1;
                const uint32_t ulo = __builtin_amdgcn_readlane((uint32_t)U, l);
                const uint32_t uhi = __builtin_amdgcn_readlane((uint32_t)(U >> 32), l);
                const uint64_t ul = ((uint64_t)uhi << 32) | ulo;
                if (lane == (uint32_t)l) {
                    const uint32_t off = (w - HW) * 64 + (uint32_t)(__ffsll((unsigned long long)ul) - 1);
                    atomicMin(&s_first[k + 1], off);
                }
                found |= 1u << (k + 1);
            }
        }
        if (U) {
            // still unresolved after the in-LDS steps: exact tail pass
            uint64_t x = U;
            while (x) {
                const int bit = __ffsll((unsigned long long)x) - 1;
                x &= x - 1;
                const unsigned long long idx = atomicAdd(&P.acc->tail_count, 1ull);
                if (idx < P.tail_cap)
                    P.tail_n[idx] = j0 + (uint64_t)bit;
                else
                    atomicOr(&P.acc->status, (unsigned)ESQ_STATUS_TAIL_OVERFLOW);
            }
        }
        if (MODE == 1 && V) {
            if (U) {
#pragma unroll
                for (int i = 0; i < 16; i++)
                    D[i] &= ~(spread4((uint32_t)(U >> (4 * i)) & 15u) * 0xffu);
            }
            store_depths(P.out_mink + ((int64_t)j0 - (int64_t)P.I0), D, V);
        }
    }

    // 4. workgroup totals -> call accumulators
#pragma unroll
    for (int k = 1; k <= kMaxKh; k++) {
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
        atomicAdd(&P.acc->cnt[tid], (unsigned long long)s_cnt[tid]);
    if (tid >= 2 && tid <= klds + 1 && s_first[tid] != kNone32)
        atomicMin(&P.acc->first[tid], (unsigned long long)(As + s_first[tid]));
}

hipError_t launch_segment(const SegParams& p, int mode, uint32_t block, hipStream_t s)
{
    const size_t lds = (size_t)p.rw * 8;
    if (p.nseg == 0)
        return hipSuccess;
    switch (mode) {
    case 0:
        hipLaunchKernelGGL(k_segment<0>, dim3(p.nseg), dim3(block), lds, s, p);
        break;
    case 1:
        hipLaunchKernelGGL(k_segment<1>, dim3(p.nseg), dim3(block), lds, s, p);
        break;
    default:
        hipLaunchKernelGGL(k_segment<2>, dim3(p.nseg), dim3(block), lds, s, p);
        break;
    }
    return hipGetLastError();
}

// --------------------------------------------------------------- tail

// Exact search, by trial division over the resident prime squares, for the
// n whose first k_lds candidates were all marked (Algorithm 2 continued).
__global__ __launch_bounds__(256) void k_tail(TailParams P)
{
    __shared__ int s_hit;
    const unsigned long long total = P.acc->tail_count;
    const uint64_t count = total < P.tail_cap ? total : P.tail_cap;
    volatile int* hitp = &s_hit;
    for (uint64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
        const uint64_t j = P.tail_n[idx];
        const uint64_t n = 2 * j + 1;
        uint32_t d = 0;
        for (uint32_t k = P.k_lds + 1; k <= 63; k++) {
            if (k > P.kmax_eff)
                break;
            const uint64_t pk = 1ull << k;
            if (pk >= n)
                break;
            const uint64_t m = n - pk;
            if (threadIdx.x == 0)
                *hitp = 0;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < P.nprimes; i += blockDim.x) {
                const uint64_t pr = P.primes[i];
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
            P.tail_d[idx] = (uint8_t)d;
            atomicAdd(&P.acc->deep_hist[d], 1ull);
            const uint32_t top = d ? d : 64u;
            for (uint32_t kk = P.k_lds + 2; kk <= top; kk++)
                atomicMin(&P.acc->first[kk], (unsigned long long)j);
            if (P.out_mink)
                P.out_mink[j - P.I0] = (uint8_t)d;
        }
    }
}

hipError_t launch_tail(const TailParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_tail, dim3(512), dim3(256), 0, s, p);
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

__global__ __launch_bounds__(1024) void k_finalize(FinParams P)
{
    extern __shared__ unsigned long long s_sort[];
    __shared__ unsigned long long s_acc;
    __shared__ unsigned int s_fill;
    const Acc* A = P.acc;
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const unsigned long long tail_total = A->tail_count;
    const uint64_t nlist = tail_total < P.tail_cap ? tail_total : P.tail_cap;
    const uint64_t n_exc = A->deep_hist[0];
    const uint64_t want = n_exc < P.exc_cap ? n_exc : P.exc_cap;

    if (P.out_exceptions && want > 0) {
        // the want-th smallest exception (binary search on its odd index)
        uint64_t thr = kNone;
        if (want < n_exc) {
            uint64_t lo = 0, hi = 1ull << 56;
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                unsigned long long c = 0;
                for (uint64_t i = tid; i < nlist; i += T)
                    c += (P.tail_d[i] == 0 && P.tail_n[i] <= mid) ? 1ull : 0ull;
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
            if (P.tail_d[i] == 0 && P.tail_n[i] <= thr) {
                const unsigned int slot = atomicAdd(&s_fill, 1u);
                if (slot < kFinalizeSortCap)
                    s_sort[slot] = P.tail_n[i];
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
            P.out_exceptions[i] = 2 * s_sort[i] + 1;
    }

    if (tid != 0)
        return;
    esq_summary* out = reinterpret_cast<esq_summary*>(P.out_summary);
    unsigned long long h[65];
    for (int k = 0; k < 65; k++)
        h[k] = 0;
    unsigned long long prev = P.n_odd;
    for (uint32_t k = 1; k <= P.k_lds; k++) {
        const unsigned long long c = A->cnt[k];
        h[k] = prev - c;
        prev = c;
    }
    for (uint32_t k = P.k_lds + 1; k < 65; k++)
        h[k] += A->deep_hist[k];
    h[0] = A->deep_hist[0];
    unsigned long long ksum = 0;
    uint32_t kseen = 0;
    for (uint32_t k = 1; k < 65; k++) {
        ksum += (unsigned long long)k * h[k];
        if (h[k])
            kseen = k;
    }
    // record-setters: first[k] = least n-index with depth >= k; each distinct
    // value is a record, labelled with the deepest level sharing it
    esq_record* rec = reinterpret_cast<esq_record*>(P.out_records);
    uint32_t nrec = 0;
    if (P.n_odd) {
        uint32_t k = 1;
        while (k <= 64) {
            const unsigned long long v = (k == 1) ? P.I0 : A->first[k];
            if (v == kNone)
                break;
            uint32_t kk = k;
            while (kk < 64 && A->first[kk + 1] == v)
                kk++;
            if (rec && nrec < ESQ_RECORDS_CAP) {
                rec[nrec].n = 2 * v + 1;
                rec[nrec].k = kk == 64 ? 0u : kk;
                rec[nrec].reserved = 0;
            }
            nrec++;
            k = kk + 1;
        }
    }
    out->n0 = P.n_odd ? 2 * P.I0 + 1 : 0;
    out->n_odd = P.n_odd;
    for (int k = 0; k < 65; k++)
        out->hist[k] = h[k];
    out->ksum = ksum;
    out->kmax_seen = kseen;
    out->n_records = nrec < ESQ_RECORDS_CAP ? nrec : ESQ_RECORDS_CAP;
    out->n_exceptions = h[0];
    out->status = A->status | (tail_total > P.tail_cap ? ESQ_STATUS_TAIL_OVERFLOW : 0u);
    out->reserved = 0;
}

hipError_t launch_finalize(const FinParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), (size_t)kFinalizeSortCap * 8, s, p);
    return hipGetLastError();
}

hipError_t configure_kernels()
{
    hipError_t e;
    const int lds_max = 160 * 1024 - 8 * 1024;
    e = hipFuncSetAttribute((const void*)k_segment<0>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_segment<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_segment<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_finalize, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(kFinalizeSortCap * 8));
    return e;
}

}  // namespace esq
