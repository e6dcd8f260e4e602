/*
 * esq.h -- C-ABI of libesq, the MI355X (gfx950) library that verifies
 * Erdos' conjecture "every odd n > 1 is a squarefree number plus a power of
 * two" on whole intervals of odd integers, after C. Hercher, "On the Sum of
 * Squarefree Integers and a Power of Two", arXiv 2411.01964.
 *
 * The signatures follow the paper's statement of the two algorithms:
 *   Algorithm 1 (Section 3): input start, end; output, for every odd number
 *     in [start, end), whether it is squarefree        -> esq_sieve_segment
 *   Algorithm 2 (Section 3): input start, end, k_max; output, for every odd n
 *     in [start, end), the least k >= 1 with n - 2^k squarefree, and a report
 *     of every n with no such k                         -> esq_verify_range
 *   "Collecting the results" (Section 3): aggregates instead of per-n arrays
 *     (maximum k, sum of k), and the per-k counts and record-setters of
 *     Section 4 (Tables 3 and 4)                        -> esq_summary
 *
 * Conventions shared by every entry point
 *   - Ranges are half-open, [lo, hi).  Odd numbers only.  esq_verify_range
 *     examines the odd n >= 3 (the conjecture concerns n > 1); the candidate
 *     m = n - 2^k must satisfy m >= 1, i.e. 2^k < n, and k >= 1 (k = 0 is
 *     excluded, so m is odd).  1 counts as squarefree.
 *   - Device memory: every pointer argument marked "device" must be
 *     device-accessible memory (hipMalloc'd, a torch CUDA tensor, or pinned
 *     host memory from hipHostMalloc).  The caller owns and frees every
 *     output buffer; the library never frees caller memory.  The library owns
 *     the resident prime table, the pattern table and per-call scratch.
 *     Scratch comes from blocks the library keeps for reuse (at most 16,
 *     4 GiB in all, per device, held until esq_shutdown): a call takes the
 *     block its stream used last, or another one after making its stream
 *     wait (on the device) for that block's last use; when none serves, or
 *     the stream is capturing a graph, it is allocated and released in stream
 *     order from a memory pool on the caller's stream.
 *   - Asynchrony: calls only enqueue work on `stream` (a hipStream_t; NULL =
 *     the default stream) and return.  Outputs are valid once the stream has
 *     been synchronised.  Calls on different streams may overlap.
 *   - Errors: 0 on success, a negative ESQ_E* code otherwise (nothing is
 *     enqueued then); esq_last_error() gives a message for the calling thread.
 *     Conditions that only the device can see are reported in
 *     esq_summary.status (ESQ_STATUS_* bits) once the stream has finished.
 */
#ifndef ESQ_H
#define ESQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define ESQ_OK 0
#define ESQ_EINVAL (-1)    /* bad argument (null required pointer, kmax > 63, lo > hi, ...) */
#define ESQ_ERANGE (-2)    /* hi above the bound given to esq_init */
#define ESQ_ENOMEM (-3)    /* device or host allocation failed */
#define ESQ_EHIP (-4)      /* a HIP runtime call failed */
#define ESQ_ENOINIT (-5)   /* esq_init has not been called (or failed) */

/* esq_summary.status bits, set by the device */
#define ESQ_STATUS_TAIL_OVERFLOW 1u  /* more unresolved n than the tail capacity:
                                        counts past the in-LDS depth and the
                                        exception list are incomplete */
#define ESQ_STATUS_BUCKET_OVERFLOW 2u /* internal bound on large-prime hits
                                         exceeded (never expected) */
#define ESQ_STATUS_EXCEPTIONS_INCOMPLETE 4u /* kmax <= the in-LDS depth and more
                                               exceptions than the tail capacity:
                                               every count is exact, the list of
                                               exceptions may miss some */

/* esq_record.flags bits */
#define ESQ_RECORD_KMAX_LIMIT 1u /* k = 0 record: the search stopped at kmax
                                    while 2^(kmax+1) < n, i.e. a larger k was
                                    still positive; 0 = every k with 2^k < n
                                    was tried and failed */

#define ESQ_MAX_HI (((uint64_t)1) << 56) /* largest hi accepted by esq_init */
#define ESQ_RECORDS_CAP 64               /* capacity of out_records per call */
#define ESQ_EXCEPTIONS_CAP_MAX 16384     /* largest exceptions_cap accepted */
#define ESQ_NOALLOC_SCRATCH_MAX (((uint64_t)64) << 20) /* static scratch of
                                    esq_verify_range_noalloc, per device */

/* A record-setter (Table 3 of Section 4): an odd n whose least k is strictly
 * larger than the least k of every smaller odd n of the same call.  An n with
 * no representation counts as deeper than any k: it is reported once, with
 * k = 0, and no later n of the call can be a record.  flags tells why such an
 * n has none (Algorithm 2's "no representation found" report): the search
 * limit kmax, or exhaustion of every positive n - 2^k. */
typedef struct esq_record {
    uint64_t n;
    uint32_t k;     /* least k, or 0 for an n with no representation */
    uint32_t flags; /* ESQ_RECORD_* bits; 0 unless k = 0 */
} esq_record;

/* Aggregates of one call ("Collecting the results", Section 3; Table 4). */
typedef struct esq_summary {
    uint64_t n0;           /* first odd n examined (>= 3); 0 if none */
    uint64_t n_odd;        /* number of odd n examined */
    uint64_t hist[65];     /* hist[k] = #n with least k (1..63); hist[0] = #n with none */
    uint64_t ksum;         /* sum of least k over the n that have one */
    uint32_t kmax_seen;    /* largest least k found (0 if none) */
    uint32_t n_records;    /* number of record-setters (<= ESQ_RECORDS_CAP) */
    uint64_t n_exceptions; /* = hist[0]; may exceed the exceptions capacity */
    uint32_t status;       /* ESQ_STATUS_* bits; 0 = complete and exact */
    uint32_t reserved;
} esq_summary;

/*
 * Select HIP device `device` and make the library resident on it: the odd
 * primes p <= isqrt(max_hi) (Algorithm 1's prime list, Section 3) and two
 * periodic tables of the odd multiples of 9, 25, 49 and of 121, 169.
 * Idempotent; a larger max_hi extends the prime table.  max_hi <= ESQ_MAX_HI.
 * Synchronous.
 */
int esq_init(int device, uint64_t max_hi);

/*
 * Algorithm 1 (Section 3) alone: squarefree flags of the odd m in [lo, hi).
 * d_bits (device, caller-owned) receives ceil(n/64) little-endian uint64
 * words, n = number of odd m in [max(lo,1), hi): bit i (LSB first) of the
 * stream is 1 iff m0 + 2i is squarefree, m0 = first odd >= max(lo, 1).  Bits
 * past the last m are 0.  hi <= the max_hi given to esq_init.  d_bits needs
 * 8-byte alignment; at 16-byte alignment whole segments go out with 16-byte
 * stores.
 */
int esq_sieve_segment(uint64_t lo, uint64_t hi, uint64_t *d_bits, void *stream);

/*
 * Algorithm 2 (Section 3) over every odd n in [lo, hi) with n >= 3, and the
 * aggregates of "Collecting the results".
 *   kmax           search limit: k runs 1, 2, ... while 2^k < n and
 *                  (kmax == 0 or k <= kmax).  0 = no limit other than
 *                  positivity.  kmax <= 63.
 *   d_out_mink     device, nullable; n_odd bytes: [i] = least k of n0 + 2i,
 *                  0 where none was found.  Any alignment; no byte outside
 *                  the n_odd is written.
 *   out_summary    device, required: one esq_summary.
 *   out_records    device, nullable: ESQ_RECORDS_CAP entries; the first
 *                  n_records are the record-setters in ascending n.
 *   out_exceptions device, nullable when exceptions_cap == 0: the smallest
 *                  min(exceptions_cap, n_exceptions) n with no representation,
 *                  ascending.  exceptions_cap <= ESQ_EXCEPTIONS_CAP_MAX.
 * Every count in the summary is exact unless status says otherwise.
 */
int esq_verify_range(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t *d_out_mink,
                     esq_summary *out_summary, esq_record *out_records,
                     uint64_t *out_exceptions, uint64_t exceptions_cap, void *stream);

/*
 * esq_verify_range for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as esq_verify_range; the
 * call allocates nothing (no hipMalloc/hipFree, no memory pool, no staging
 * buffer, no event).  Its scratch (per-interval accumulators, large-prime
 * hit slots, the list of n left to the exact tail pass) is a static device
 * array of ESQ_NOALLOC_SCRATCH_MAX bytes that every device the library runs
 * on holds from esq_init until the process ends.
 *   - Returns ESQ_ERANGE, enqueuing nothing, when the interval needs more
 *     scratch than that (esq_scratch_bytes with count = 1 gives the figure;
 *     about 26 MB for 2^33 odd n near 2^50 with the default knobs), and
 *     ESQ_ENOMEM when the medium-prime tables of the current knobs are not
 *     resident (esq_init and esq_set_param make them).
 *   - Every call on one device uses the same array and clears what must
 *     start at zero on the device: calls that overlap in time on one device
 *     (different streams, or threads) race and give wrong results.  Serialise
 *     them, e.g. on one stream.
 */
int esq_verify_range_noalloc(uint64_t lo, uint64_t hi, uint32_t kmax, uint8_t *d_out_mink,
                             esq_summary *out_summary, esq_record *out_records,
                             uint64_t *out_exceptions, uint64_t exceptions_cap, void *stream);

/*
 * Many intervals in one launch (the batched form of esq_verify_range): every
 * interval [lo[i], hi[i]) is cut into segments, and persistent workgroups
 * pull runs of consecutive segments of any interval from one device work
 * queue, so short and long intervals share the GPU.  Results per interval are
 * identical to esq_verify_range on that interval alone.
 *   count          number of intervals
 *   lo, hi         host arrays of count bounds (half-open, as above)
 *   kmax           as in esq_verify_range, for every interval
 *   d_out_mink     host array of count device pointers (entries may be NULL)
 *                  receiving each interval's per-n least k; or NULL
 *   out_summaries  device, required: count esq_summary
 *   out_records    device, nullable: count * ESQ_RECORDS_CAP esq_record;
 *                  interval i's records start at i * ESQ_RECORDS_CAP
 * Exceptions are counted (hist[0]) but not listed.
 */
int esq_verify_batch(uint32_t count, const uint64_t *lo, const uint64_t *hi, uint32_t kmax,
                     uint8_t *const *d_out_mink, esq_summary *out_summaries,
                     esq_record *out_records, void *stream);

/*
 * Device scratch, in bytes, that one esq_verify_batch call over these
 * intervals holds while it runs (a kept block or pool memory): per-segment
 * hit slots of the large primes, the list of n left to the exact tail pass,
 * per-interval descriptors and accumulators.  The caller's outputs
 * (summaries, records, per-n bytes) are not included.  For count = 1 it is
 * also the scratch of esq_verify_range on that interval with
 * exceptions_cap = 0.  For admission control by a server: a request is
 * admitted when its scratch and its outputs fit in device memory.
 *   count, lo, hi, kmax  as in esq_verify_batch (host arrays)
 *   out_bytes            host, required
 * Synchronous; enqueues nothing.  Errors as esq_verify_batch.
 */
int esq_scratch_bytes(uint32_t count, const uint64_t *lo, const uint64_t *hi, uint32_t kmax,
                      uint64_t *out_bytes);

/*
 * Prepared batches: the same work as esq_verify_batch, planned once, with its
 * scratch and descriptors kept on the device, so that it can be launched
 * repeatedly without host planning, allocation or copies -- and captured as
 * a hipGraph.
 *   esq_batch_create   plans and allocates (synchronous); the output pointers
 *                      are bound to the handle and rewritten by every launch.
 *   esq_batch_launch   enqueues the kernels on `stream`; with use_graph != 0
 *                      the kernel sequence is captured into a hipGraph on the
 *                      first such launch and replayed afterwards.  Launches of
 *                      one handle must not overlap in time (they share its
 *                      scratch); different handles may run concurrently.
 *   esq_batch_destroy  waits for the device and frees the handle.
 */
typedef struct esq_batch esq_batch;
/* A prepared batch holds the library's resident tables: esq_batch_launch
 * returns ESQ_EINVAL, launching nothing, once esq_init has replaced them (a
 * larger max_hi, another device) or esq_shutdown has released them. */
int esq_batch_create(uint32_t count, const uint64_t *lo, const uint64_t *hi, uint32_t kmax,
                     uint8_t *const *d_out_mink, esq_summary *out_summaries,
                     esq_record *out_records, esq_batch **out_handle);
int esq_batch_launch(esq_batch *batch, int use_graph, void *stream);
void esq_batch_destroy(esq_batch *batch);

/*
 * Tuning knobs (results never depend on them; only speed does).  Names:
 *   "seg_log2"   log2 of the segment length in odd numbers held in LDS (10..20)
 *   "sieve_seg_log2" the same for esq_sieve_segment (default 20: one
 *                workgroup per CU whose storer waves write the bitmap while
 *                its loader waves start the next segment)
 *   "kh"         deepest k resolved from the LDS bitmap (1..13); deeper k go
 *                to the exact tail pass
 *   "block"      threads per workgroup of the segment kernel, summary mode
 *                (64..1024, x64; default 512)
 *   "per_n_block" the same in per-n mode for one interval (default 1024;
 *                per-n batches of several intervals use "block")
 *   "sieve_block" the same for esq_sieve_segment (default 1024)
 *   "entry_hits" target marks per lane-task for medium primes (1..4096)
 *   "tail_cap"   capacity of the per-call list of n unresolved in LDS
 *   "profile"    1 = time each segment-kernel launch (esq_profile_take)
 *   "phase_clock" 1 = count the segment kernel's time per phase
 *                (esq_phase_take); costs a few atomics per segment
 *   "medium_max" largest prime whose multiples every segment marks itself
 *                (11..11000); larger primes go through per-segment hit slots
 *   "bucket_cap" hit slots per segment (0 = sized from the expected count);
 *                a segment whose slots overflow marks those primes directly
 *   "items_per_wg" batched form: work items (runs of consecutive segments)
 *                per resident workgroup
 *   "runs_per_wg" single interval: runs of consecutive segments per resident
 *                workgroup (1..64)
 *   "stagger"    segment kernel, summary mode: start delay of each
 *                later-launched quarter of the workgroups, in units of 64
 *                clocks (0..4096; 0 = none; default 72, about a quarter of a
 *                segment at seg_log2 18)
 *   "cof_weight" large primes: the cost of one cofactor-enumeration thread in
 *                percent of one first-hit thread, in the per-launch choice of
 *                the cut-over between the two (1..10000)
 *   "priority"   segment kernel: 1 = raise the wave priority of workgroups
 *                with more of their run left (default), 0 = off
 * Applies to calls made after it.  Returns ESQ_EINVAL for an unknown name
 * or a value out of range.
 */
int esq_set_param(const char *name, int64_t value);
int64_t esq_get_param(const char *name); /* -1 for an unknown name */

/*
 * Kernel timing for measurement.  While the knob "profile" is 1, every call
 * records a pair of HIP events on its own stream around its segment-kernel
 * launch (the kernel that sieves and searches in LDS).  esq_profile_take
 * waits for the recorded events, writes the summed kernel time in
 * milliseconds and the number of launches since the previous take, and
 * clears the record.  Host pointers.  Returns ESQ_EINVAL for null pointers.
 */
int esq_profile_take(double *total_ms, uint64_t *launches);

/*
 * Phase clock for measurement.  While the knob "phase_clock" is 1, the
 * segment kernel adds, per workgroup and segment, the time from the segment's
 * start to the end of its wheel init, of its marking (Algorithm 1), and of
 * its search (Algorithm 2) or bitmap store, in ticks of the device's
 * constant-rate counter (100 MHz on MI355X).  esq_phase_take waits for the
 * device, writes the three sums to ticks (host, 3 values) and clears them.
 * Returns ESQ_EINVAL for a null pointer, ESQ_ENOINIT before esq_init.
 */
int esq_phase_take(uint64_t *ticks);

/*
 * Measured ceilings of the current device, for the rooflines of the segment
 * kernel (Section 3's sieve is LDS work, its search VALU work, the pattern
 * init L2 reads, the per-n and sieve outputs HBM writes): microbenchmarks of
 * conflict-free LDS operations, of int32 VALU issue, of L2 reads (eight
 * 256-thread workgroups per CU) and of HBM writes (one 16-byte store per
 * thread over the buffer), best of three timed launches each.  out (host,
 * ESQ_CEILINGS doubles) receives:
 * [0] ds_write_b64 bytes/s, [1] ds_read_b64 bytes/s, [2] ds_or_b32 bytes/s,
 * int32 VALU lane-operations/s of [3] v_add_u32/v_xor_b32, [4] v_alignbit_b32,
 * [5] v_bcnt_u32_b32, [6] L2 read bytes/s of 16-byte loads over a 1 MiB
 * buffer, and [7] HBM write bytes/s of 16-byte stores streaming over 2 GiB.
 * Synchronous; allocates and frees device buffers (2 GiB at most).  Returns
 * ESQ_EINVAL for a null pointer, ESQ_ENOMEM or ESQ_EHIP on a HIP failure.
 */
#define ESQ_CEILINGS 8
int esq_measure_ceilings(double *out);

/* Message for the last non-zero return on the calling thread ("" if none). */
const char *esq_last_error(void);

/* Release every device resource.  esq_init may be called again afterwards. */
void esq_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* ESQ_H */
