// Internal declarations shared by the kernels (esq_kernels.hip) and the
// host library (esq_api.hip).  Not part of the public C-ABI.
//
// Coordinates.  Odd numbers are addressed by their "odd index"
// i(m) = (m - 1) / 2, so m = 2i + 1.  For odd n, n - 2^k has odd index
// i(n) - 2^(k-1): the k-th candidate of Algorithm 2 (Section 3) sits
// 2^(k-1) bits below n in a bitmap over odd numbers.  The odd multiples of
// p^2 are p^2 (2t + 1), i.e. the odd indices congruent to (p^2 - 1) / 2
// modulo p^2 -- spaced p^2 apart, as Algorithm 1 steps by 2 p^2 in integers.
//
// A segment covers S = 2^log2S consecutive odd indices (its "main" part)
// plus hlo_words * 64 indices below it (the halo, so that candidates of the
// segment's n up to depth kh fall inside LDS) and hup_words * 64 above it.
// Bitmap bits are 1 for "not squarefree or not a positive odd number".
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esq {

constexpr uint32_t kWheelPeriod = 9u * 25u * 49u * 121u;  // 1334025
constexpr uint32_t kWheelExtra = 16640;   // >= largest region in 64-bit words
constexpr int kMaxKh = 13;                // deepest in-LDS level supported
constexpr int kMaxMedium = 512;           // medium primes per segment (LDS table)
constexpr unsigned long long kNone = ~0ull;
constexpr uint32_t kNone32 = ~0u;
constexpr int kMaxSegLog2 = 20;
constexpr int kMinSegLog2 = 10;
constexpr uint32_t kFinalizeSortCap = 16384;  // LDS sort capacity of the finalize pass

// Per-call accumulators in device scratch.
struct Acc {
    unsigned long long cnt[65];        // cnt[k]: #n still unresolved after step k (k <= k_lds)
    unsigned long long first[65];      // first[k]: least n-index with depth >= k
    unsigned long long deep_hist[65];  // tail pass: [0] no representation, [k] least k
    unsigned long long tail_count;     // #n unresolved after the in-LDS steps
    unsigned int status;               // ESQ_STATUS_* bits
    unsigned int bucket_total;
};

struct MedEntry {   // one lane-task of the medium-prime marking
    uint32_t idx;   // medium prime index (0 = the prime 13)
    uint32_t vc;    // v | (c << 16): marks f + (v + c t) q for t >= 0
};

struct SegParams {
    int64_t A0;             // odd index of segment 0's first main bit (multiple of 64)
    uint32_t log2S;         // main length S = 2^log2S
    uint32_t hlo_words;     // halo below, in 64-bit words
    uint32_t rw;            // region words = hlo_words + S/64 + hup_words
    uint32_t nseg;
    uint32_t wheel_base0;   // floor((A0 - 64 hlo_words) / 64) mod kWheelPeriod
    uint32_t wheel_step;    // (S / 64) mod kWheelPeriod
    const uint64_t* wheel;  // kWheelPeriod + kWheelExtra words
    const uint32_t* primes; // odd primes, ascending
    uint32_t med_begin;     // index of 13 in primes
    uint32_t nmed;          // medium primes: primes[med_begin .. med_begin + nmed)
    const MedEntry* med;    // lane-tasks
    uint32_t n_med_entries;
    uint32_t pad0;
    const uint32_t* bucket_off;  // nseg + 1 offsets, or null
    const uint32_t* bucket_ent;  // region bit offsets of large-prime hits
    uint64_t bucket_cap;         // entries allocated
    // verification
    uint64_t I0, I1;        // odd indices of the n examined: [I0, I1)
    uint32_t k_lds;         // steps resolved from LDS (<= kMaxKh)
    uint32_t pad1;
    Acc* acc;
    unsigned long long* tail_n;
    uint64_t tail_cap;
    uint8_t* out_mink;      // per-n bytes, indexed by n-index - I0, or null
    // sieve output (Algorithm 1 alone)
    uint64_t* out_bits;
    uint64_t n_bits;        // bits of output
    uint32_t out_shift;     // I0 - A0
    uint32_t pad2;
};

struct BucketParams {
    const uint32_t* primes;
    uint32_t p_begin;       // first bucket prime (index)
    uint32_t n_heavy;       // primes [p_begin, p_begin + n_heavy): one workgroup each
    uint32_t n_light;       // then one thread each
    uint32_t log2S;
    uint32_t overlap;       // region length - S (segment regions overlap by this much)
    uint32_t nseg;
    int64_t B0;             // odd index of segment 0's region start
    uint64_t E;             // extent of all regions, y in [0, E)
    uint32_t* counts;       // nseg
    uint32_t* cursor;       // nseg
    const uint32_t* offsets;  // nseg + 1
    uint32_t* entries;
    uint64_t capacity;
    Acc* acc;
};

struct TailParams {
    Acc* acc;
    const unsigned long long* tail_n;
    uint8_t* tail_d;
    uint64_t tail_cap;
    const uint32_t* primes;
    uint32_t nprimes;
    uint32_t k_lds;
    uint32_t kmax_eff;
    uint32_t pad;
    uint64_t I0;
    uint8_t* out_mink;
};

struct FinParams {
    const Acc* acc;
    const unsigned long long* tail_n;
    const uint8_t* tail_d;
    uint64_t tail_cap;
    uint64_t n_odd;
    uint64_t I0;
    uint32_t k_lds;
    uint32_t pad;
    void* out_summary;          // esq_summary
    void* out_records;          // esq_record[64] or null
    uint64_t* out_exceptions;   // or null
    uint64_t exc_cap;
};

// launchers (esq_kernels.hip); all return hipError_t of the launch
hipError_t launch_wheel_build(uint64_t* wheel, hipStream_t s);
hipError_t launch_prepare(Acc* acc, uint32_t* counts, uint32_t* cursor, uint32_t nseg,
                          hipStream_t s);
hipError_t launch_bucket(const BucketParams& p, bool fill, hipStream_t s);
hipError_t launch_scan(const uint32_t* counts, uint32_t* offsets, uint32_t nseg, Acc* acc,
                       uint64_t capacity, hipStream_t s);
hipError_t launch_segment(const SegParams& p, int mode, uint32_t block, hipStream_t s);
hipError_t launch_tail(const TailParams& p, hipStream_t s);
hipError_t launch_finalize(const FinParams& p, hipStream_t s);
hipError_t configure_kernels();

}  // namespace esq
