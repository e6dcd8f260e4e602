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
//
// Work is a list of intervals; each interval is cut into segments, and runs
// of consecutive segments ("items") are pulled by persistent workgroups from
// a device queue.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esq {

constexpr uint32_t kWheelPeriod = 9u * 25u * 49u;  // 11025 words: the table stays in L2
constexpr uint32_t kWheelExtra = 16640;   // >= largest region in 64-bit words
constexpr uint32_t kWheel2Period = 121u * 169u;  // 20449 words: second table (11^2, 13^2)
constexpr size_t kWheelAlloc = 2u << 20;  // bytes holding both tables, at both origins
constexpr uint32_t kFirstMedium = 5;      // primes[0 .. 5) = 3, 5, 7, 11, 13: the two tables
constexpr int kMaxKh = 13;                // deepest in-LDS level supported
constexpr int kMaxMedium = 1536;          // medium primes per launch (LDS offsets)
constexpr unsigned long long kNone = ~0ull;
constexpr int kMaxSegLog2 = 20;
constexpr uint32_t kFlushSegs = 4096;     // segments per run and per flush of partial totals
constexpr int kMinSegLog2 = 10;
constexpr uint32_t kFinalizeSortCap = 16384;  // LDS sort capacity of the finalize pass
constexpr uint32_t kPidxShift = 8;        // coarse prime index: 256 integers per entry
constexpr uint64_t kCofactorPrime = 1u << 20; // largest direct/cofactor cut-over considered

// Per-interval accumulators in device scratch.
struct Acc {
    unsigned long long cnt[16];        // cnt[k]: #n still unresolved after step k (k <= k_lds)
    unsigned long long first[65];      // first[k]: least n-index with depth >= k
    unsigned long long deep_hist[65];  // tail pass: [0] no representation, [k] least k
    unsigned long long tail_count;     // #n of this interval sent to the tail pass
    unsigned int status;               // ESQ_STATUS_* bits
    unsigned int pad;
};

// One interval of a launch.
struct Interval {
    int64_t A0;             // odd index of segment 0's first main bit (multiple of 64)
    uint64_t I0, I1;        // verify: odd indices of the n examined; sieve: of the output bits
    uint32_t nseg;          // segments
    uint32_t seg_base;      // global index of segment 0 (bucket slots)
    uint32_t wheel_base0;   // floor((A0 - 64 hlo_words) / 64) mod kWheelPeriod
    uint32_t pmax_end;      // primes[0 .. pmax_end) are all the primes this interval needs
    uint32_t b_direct_end;  // bucket primes by first hit: primes[med_end .. b_direct_end)
    uint32_t n_cof;         // odd cofactors j = 1, 3, ... for primes from b_direct_end on
    Acc* acc;
    uint8_t* out_mink;      // per-n bytes (n-index - I0), or null
    uint64_t* out_bits;     // sieve output words, or null
    uint32_t out_shift;     // sieve: I0 - A0
    uint32_t n_cof_wide;    // the first n_cof_wide cofactors (widest ranges) take 8 lanes each
};

// Medium-prime lane-task, packed in a uint2: x = v q | (idx << 21), y = c q;
// it marks f + v q + t c q, t >= 0, of medium prime idx (0 = the prime 17),
// f its first hit in the region.

// Geometry and resources shared by every interval of a launch.
struct Launch {
    uint32_t log2S;
    uint32_t hlo_words, hup_words, rw;  // rw = hlo_words + S/64 + hup_words
    uint32_t n_iv;                // intervals
    uint32_t n_items;             // work items in the queue
    uint32_t stage;               // per-n mode: depth bytes staged through LDS per wave
    uint32_t mode;                // 0 verify, 1 verify + per-n, 2 sieve
    uint32_t med_end;             // medium primes primes[kFirstMedium .. med_end)
    uint32_t n_tasks;
    uint32_t k_lds, kmax_eff;     // k_lds >= kmax_eff: every n unresolved in LDS is an exception
    uint32_t exc_list;            // 1: the call lists its exceptions (single interval)
    uint32_t bucket_cap;          // hit slots per segment
    uint32_t nprimes;
    const Interval* iv;
    const uint4* items;           // (interval, first segment, segments, 0), or null
    const uint32_t* primes;       // odd primes ascending
    const uint32_t* pidx;         // pidx[v]: index of the first prime >= v << kPidxShift
    uint32_t pidx_n;              // entries of pidx
    const uint64_t* qinv;         // qinv[i] = floor(2^64 / primes[i]^2) for i < n_qinv
    uint32_t n_qinv;              // every prime <= kCofactorPrime has one
    const uint2* medq;            // per medium prime: (q, S mod q)
    const uint2* tasks;           // medium-prime lane-tasks
    uint32_t tasks_in_lds;        // 1: the task table is copied into LDS
    uint32_t stagger;             // start delay per workgroup slot, in units of 64 clocks (0: none)
    uint32_t priority;            // 1: wave priority from the share of the run left
    unsigned long long* phase;    // non-null: per-phase clock ticks of the segment loop (init, marking, search or store, segments)
    const uint64_t* wheel;        // kWheelPeriod + kWheelExtra words (9, 25, 49)
    const uint64_t* wheel2;       // kWheel2Period + kWheelExtra words (121, 169)
    uint32_t origin;              // 1: a region's bit 0 is the odd index one below its word
                                  // boundary (search modes; wheel tables shifted to match)
    uint32_t* bucket_cnt;         // per global segment
    uint32_t* bucket_slot;        // bucket_cap per global segment
    unsigned int* queue;          // work-queue head
    unsigned long long* tail_n;   // n-indices unresolved after the LDS steps
    uint32_t* tail_iv;            // their interval
    uint8_t* tail_d;              // their depth from the tail pass
    unsigned long long* tail_count;
    uint64_t tail_cap;
};

// launchers (esq_kernels.hip); all return hipError_t of the launch
hipError_t launch_wheel_build(uint64_t* wheel, uint64_t* wheel2, uint32_t shift, hipStream_t s);
hipError_t launch_prepare(const Launch& L, Acc* accs, const Interval* iv_single,
                          uint32_t nseg_total, hipStream_t s);
hipError_t launch_bucket(const Launch& L, uint32_t n_heavy, uint32_t max_direct, uint32_t max_cof,
                         hipStream_t s);
hipError_t launch_verify(const Launch& L, uint32_t grid, uint32_t block, hipStream_t s);
hipError_t launch_tail(const Launch& L, hipStream_t s);
hipError_t launch_finalize(const Launch& L, void* out_summaries, void* out_records,
                           uint64_t* out_exceptions, uint64_t exc_cap, hipStream_t s);
hipError_t configure_kernels();
int verify_occupancy(int mode, uint32_t block, size_t lds_bytes);
size_t verify_lds_bytes(const Launch& L, uint32_t block);
constexpr size_t kVerifyLdsMax = 159 * 1024;  // dynamic LDS per workgroup
constexpr uint32_t kVerifyCtrlWords = 28;       // k_verify's LDS control block, in 8-byte words
constexpr uint32_t kPhaseSlots = 8;             // phase-clock counters (3 used)
constexpr uint32_t kStageWordsPerWave = 528;    // per-n mode: one wave's 4096 depth bytes + 2 x 64 B guard

// k_verify's dynamic LDS, in 8-byte words: the region bitmap (rw), the
// control block, the medium primes' (q, S mod q) and first-hit offsets, the
// task table when it is held in LDS, and -- when per-n output is staged -- a
// store-staging area of kStageWordsPerWave words per wave, 16-byte aligned.
__host__ __device__ inline size_t verify_stage_word(uint32_t rw, uint32_t nmed, uint32_t n_tasks_lds)
{
    return ((size_t)rw + kVerifyCtrlWords + nmed + (nmed + 1) / 2 + n_tasks_lds + 1) & ~(size_t)1;
}
__host__ __device__ inline size_t verify_lds_size(uint32_t rw, uint32_t nmed, uint32_t n_tasks_lds,
                                                  bool stage, uint32_t block)
{
    if (stage)
        return (verify_stage_word(rw, nmed, n_tasks_lds) + (size_t)(block / 64) * kStageWordsPerWave) * 8;
    return ((size_t)rw + kVerifyCtrlWords + nmed + (nmed + 1) / 2 + n_tasks_lds) * 8;
}

}  // namespace esq
