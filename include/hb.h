/*
 * hb.h -- C ABI of libhb, MI355X (gfx950) batch hashing: MD5, SHA-1 and SM3 digests of
 * very many independent messages.
 *
 * The operation is the paper's multi-message ("parallel scenario") crypto op: many
 * digests computed at once, each message and each digest in its own slot so the work is
 * free of races (Sec. IV-B; Sec. V-D).  The digests themselves are defined by the
 * standards the paper names: MD5 = RFC 1321, SHA-1 = FIPS 180-4, SM3 = GB/T 32905-2016.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every function returns an int status (HB_OK or a negative HB_E* code) and
 *    never throws.  Argument errors are reported before anything is enqueued; the text of
 *    the last error on the calling thread is available from hb_last_error().
 *  - Execution is asynchronous on the given HIP stream (a hipStream_t passed as void*;
 *    NULL means the legacy default stream), like hipMemcpyAsync.  A device fault surfaces
 *    as HB_EHIP from a later call or synchronisation.
 *  - Messages are bytes.  Message i is messages[offsets[i] .. offsets[i] + lengths[i]):
 *    offsets may have any byte alignment, messages may overlap or leave gaps, and a length
 *    of 0 is valid.  Lengths are below 2^61 bytes (the bit length must fit 64 bits).
 *  - Digests are the canonical digest bytes (what the standards print): 16 bytes for MD5,
 *    20 for SHA-1, 32 for SM3, digest i at digests_out + i * stride.  digests_out must be
 *    4-byte aligned, must not overlap the inputs, and stride must be a multiple of 4 and
 *    at least the digest size.  Bytes of a slot past the digest size are written as zero.
 *  - Pointers named "device" are device memory (hipMalloc / torch CUDA tensors) owned by
 *    the caller, which keeps them valid and unmodified until the stream work completes.
 *    Pointers named "host" are host memory, also owned by the caller.
 */
#ifndef HB_H
#define HB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HB_MD5 = 0, HB_SHA1 = 1, HB_SM3 = 2 };
enum { HB_OK = 0, HB_EINVAL = -1, HB_ENOMEM = -2, HB_EHIP = -3, HB_EBUDGET = -4, HB_EBUSY = -5,
       HB_ECANCELED = -6 };

/* Digest size in bytes of algo (16, 20 or 32); 0 for an unknown id. */
size_t hb_digest_size(int algo);

/* Thread-local text describing the last non-OK status returned on this thread. */
const char *hb_last_error(void);

/* Library and device facts: CU count, wave size, peak engine clock (kHz) and gfx arch
 * name of the current device.  Returns HB_EHIP if no device is visible. */
int hb_device_info(int *cu_count, int *wave_size, int *clock_khz, char *arch_name, size_t arch_len);

/*
 * hb_probe_valu -- measures the integer-VALU issue rate of the current device, the figure
 * the roofline's peak rests on (a calibration for the bench, not a hashing call).  Every CU
 * is filled with waves_per_simd workgroups of four waves; each wave runs long chains of one
 * instruction kind over eight independent accumulators per lane, or, for the compression
 * kinds, the library's own MD5 / SHA-1 / SM3 compression on register data with no memory
 * traffic (plus one xor per block feeding the state back into the words).
 *   kind            HB_PROBE_*: ADD3 v_add3_u32, ALIGNBIT v_alignbit_b32, BITOP3
 *                   v_bitop3_b32, ADD v_add_u32 (VOP2), XOR v_xor_b32 (VOP2), XAD v_xad_u32,
 *                   PERM v_perm_b32, MIX_ALT bitop3 and alignbit alternating, MIX_2_1 two
 *                   bitop3 to one alignbit, MD5 / SHA1 / SM3 compressions
 *   waves_per_simd  1..8
 *   cycles_out      host: SIMD cycles per wave instruction (instruction kinds) or per wave
 *                   and 64-byte block (compression kinds), best of three launches
 *   clock_ghz_out   host, may be null: the engine clock the waves ran at
 * Allocates a small device buffer, synchronises the device and frees the buffer: run it
 * alone.  Returns HB_EINVAL for an unknown kind, waves_per_simd outside 1..8 or a null
 * cycles_out, HB_EHIP on a HIP failure.
 */
enum { HB_PROBE_ADD3 = 0, HB_PROBE_ALIGNBIT = 1, HB_PROBE_BITOP3 = 2, HB_PROBE_ADD = 3, HB_PROBE_XOR = 4,
       HB_PROBE_XAD = 5, HB_PROBE_PERM = 6, HB_PROBE_MIX_ALT = 7, HB_PROBE_MIX_2_1 = 8, HB_PROBE_MD5 = 9,
       HB_PROBE_SHA1 = 10, HB_PROBE_SM3 = 11, HB_PROBE_KINDS = 12 };
int hb_probe_valu(int kind, int waves_per_simd, double *cycles_out, double *clock_ghz_out);

/*
 * hash_batch -- plain batch hashing, one GPU lane per message, in index order.
 *   algo         HB_MD5 / HB_SHA1 / HB_SM3
 *   messages     device, packed message bytes
 *   offsets      device, n x uint64 byte offsets into messages
 *   lengths      device, n x uint64 message lengths in bytes
 *   n            message count; 0 is a no-op returning HB_OK
 *   digests_out  device, n slots of hb_digest_size(algo) bytes (stride = digest size)
 *   stream       hipStream_t
 * Allocates nothing, so it may be captured in a hipGraph.  The padding and the length
 * field (RFC 1321 Sec. 3.1-3.2, FIPS 180-4 Sec. 5.1.1, GB/T 32905 Sec. 5.2) are built in
 * registers; no padded copy of the input is made.
 */
int hash_batch(int algo, const uint8_t *messages, const uint64_t *offsets, const uint64_t *lengths,
               uint64_t n, uint8_t *digests_out, void *stream);

/* As hash_batch, with an explicit digest stride in bytes (multiple of 4, >= digest size). */
int hash_batch_strided(int algo, const uint8_t *messages, const uint64_t *offsets,
                       const uint64_t *lengths, uint64_t n, uint8_t *digests_out,
                       uint64_t stride, void *stream);

/*
 * hash_batch_fixed -- n messages of exactly msg_len bytes stored back to back:
 * message i is messages[i * msg_len .. (i + 1) * msg_len).  No metadata arrays are read.
 * digests_out holds n slots of hb_digest_size(algo) bytes.  Allocates nothing.  When
 * messages and msg_len are multiples of 4 and msg_len < 2^25, each wave of 64 messages
 * stages two blocks of all 64 at a time through LDS with whole-line loads (HB_PLAIN_LDS=0
 * reads each lane's message on its own instead); either way the digests are the same.
 */
int hash_batch_fixed(int algo, const uint8_t *messages, uint64_t n, uint64_t msg_len,
                     uint8_t *digests_out, void *stream);

/*
 * hash_batch_mixed -- each message with its own algorithm, plain form: one launch per
 * algorithm present, each lane skipping messages of the other algorithms.
 *   algos        device, n x uint8 algorithm ids
 *   digests_out  device, n slots of 32 bytes (bytes past the digest size are zeroed)
 * An invalid id in algos is not detected on the device; its slot is left all zero.
 * Allocates nothing.
 */
int hash_batch_mixed(const uint8_t *algos, const uint8_t *messages, const uint64_t *offsets,
                     const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream);

/*
 * hash_digits9 -- the paper's own workload (Sec. V-A.2): the digests of the 9-character
 * decimal strings "000000000" .. "999999999".  Message i is the zero-padded decimal text
 * of start + i; the text is generated on the device, so no input buffer exists.
 *   start, n     0 <= start, start + n <= 10^9
 *   digests_out  device, n slots of hb_digest_size(algo) bytes
 * Allocates nothing.
 */
int hash_digits9(int algo, uint64_t start, uint64_t n, uint8_t *digests_out, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Incremental hashing: per-message chaining state between launches.                      */
/* ------------------------------------------------------------------------------------ */

/*
 * Chaining state of one message being hashed in pieces (the paper's single-message op and
 * its multi-message form, Sec. IV-B, split over several launches).  h[] holds the chaining
 * value words (MD5 4, SHA-1 5, SM3 8; the rest unused), bytes the number of message bytes
 * absorbed so far, flags 1 if an update piece was not a whole number of 64-byte blocks.
 * States live in device memory; they may be copied out and back in to suspend and resume.
 */
typedef struct hb_state {
    uint32_t h[8];
    uint64_t bytes;
    uint64_t flags;
} hb_state;

/* Set n device states to the algorithm's initial value (RFC 1321 Sec. 3.3, FIPS 180-4
 * Sec. 5.3.1, GB/T 32905 Sec. 4.1).  states: device, 8-byte aligned. */
int hash_init_batch(int algo, hb_state *states, uint64_t n, void *stream);

/* Absorb piece i (messages[offsets[i] .. + lengths[i]), device) into state i.  Pieces
 * before the final one must be whole blocks: a length that is not a multiple of 64 marks
 * the state invalid (flags = 1) and is not absorbed; an invalid state ignores later
 * pieces.  Allocates nothing. */
int hash_update_batch(int algo, hb_state *states, const uint8_t *messages, const uint64_t *offsets,
                      const uint64_t *lengths, uint64_t n, void *stream);

/* Absorb the last piece i (any length, possibly 0) and the padding, whose length field
 * counts every byte absorbed by the state plus this piece; write digest i to digests_out
 * (device, n x digest size, 4-byte aligned).  States are read only.  An invalid state
 * gives an all-zero digest slot.  Allocates nothing. */
int hash_final_batch(int algo, const hb_state *states, const uint8_t *messages, const uint64_t *offsets,
                     const uint64_t *lengths, uint64_t n, uint8_t *digests_out, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Batched form: length-bucketed, longest-first, persistent fused launch in a hipGraph.  */
/* ------------------------------------------------------------------------------------ */

typedef struct hb_plan hb_plan;

enum {
    HB_PLAN_GRAPH = 1,      /* capture the pipeline in a hipGraph and replay it (default on) */
    HB_PLAN_AUTOTUNE = 2,   /* time the kernel variants on first use and cache the choice */
    HB_PLAN_NO_SORT = 4,    /* skip bucketing: lanes take messages in index order */
    HB_PLAN_NO_LONG = 8,    /* no separate long-chain path (see hb_plan_create) */
    HB_PLAN_LONG_INLINE = 16 /* long-chain work and bulk in one launch on the run's stream:
                                no side stream */
};

/*
 * hb_plan_create -- reserve device workspace for batches of up to max_n messages and
 * build the launch plan.  The plan owns its workspace (about 4 bytes per message, a fixed
 * part of about 0.6 MB, and -- unless HB_PLAN_NO_LONG -- a long-chain scratch of
 * HB_LONG_SCRATCH_MB MiB, default 1024) and, with HB_PLAN_GRAPH, a hipGraph captured on
 * first run.  Long-chain path: messages of at least HB_LONG_MIN_BLOCKS blocks (default 256,
 * i.e. about 16 KiB) have every block's schedule words computed block-parallel first, then
 * run as rounds-only chains in a high-priority kernel beside the bulk kernel (a message's
 * blocks are strictly sequential, so this shortens the critical path, not the work);
 * those the scratch cannot hold run there as ordinary chains, at most one wave per SIMD
 * (the longest by blocks x ops per block), and when the longest chain dwarfs the rest the
 * bulk kernel runs on only as many waves as finish its work in 1/HB_BULK_MARGIN (default
 * 4; 0 = all waves) of that chain's time.  With HB_PLAN_LONG_INLINE the long-chain work
 * and the bulk run in one launch on the run's own stream (the long chains' workgroups
 * first), with the same concurrency and no side stream, for callers that keep several
 * plans busy on streams of their own and have no hardware queue to spare for each; that
 * launch takes the long-chain kernel's register budget, so its bulk waves run at lower
 * occupancy.  Returns HB_ENOMEM if the workspace cannot be allocated.
 */
int hb_plan_create(hb_plan **plan, uint64_t max_n, int flags);

/*
 * hb_plan_run -- hash n <= max_n messages.  algos (device, n x uint8) gives per-message
 * algorithm ids; when algos is NULL every message uses algo.  digests_out stride is 32
 * bytes when algos != NULL, else hb_digest_size(algo).  Other arguments as hash_batch.
 * The steps (all on the device, in stream order): per-message block count
 * nb = floor((L + 8) / 64) + 1; counting sort by (algorithm, nb) descending; work items
 * of one wave each (algorithm-uniform lanes of near-equal nb); items merged by estimated
 * cost, longest first; one persistent launch whose waves pull items from an atomic queue.
 * Messages of at least HB_LONG_MIN_BLOCKS blocks take the long-chain path (see
 * hb_plan_create).  Per-run pointers and sizes reach the device through a one-thread
 * kernel launched ahead of the pipeline with them as arguments, so a captured graph is
 * replayed unchanged and consecutive runs need no host synchronisation.  Calls on one plan
 * must be serialised by the caller (a plan is not thread-safe) and one plan's runs must
 * share a stream, since they share the plan's workspace.
 */
int hb_plan_run(hb_plan *plan, const uint8_t *algos, int algo, const uint8_t *messages,
                const uint64_t *offsets, const uint64_t *lengths, uint64_t n,
                uint8_t *digests_out, void *stream);

/* Launch choices of a plan (after autotuning, if enabled): persistent-kernel waves per CU,
 * messages per lane per work item, and the message-load scheme `variant`:
 *   0  whole blocks in bursts of the default depth (MD5 four, SHA-1 / SM3 two) -- default
 *   1  SHA-1 / SM3 one block at a time with the next block's loads in flight; MD5 as 0
 *   2  one block per load
 *   3  bursts of two whole blocks for every algorithm
 *   4  bursts of four whole blocks for every algorithm
 * With HB_PLAN_AUTOTUNE the first run times waves per CU {8, 16, 32} x messages per lane
 * {1, 2} x the five schemes on its own input and keeps the fastest, cached per device, CU
 * count, algorithm mix and length bucket (mean block count and spread, read from the
 * plan's histogram); HB_TUNE_CACHE names a file that keeps the cache across processes. */
int hb_plan_config(const hb_plan *plan, int *waves_per_cu, int *msgs_per_lane, int *variant);

/* Force launch choices (0 keeps the current waves per CU / messages per lane; variant is
 * set as given, 0..4); drops any captured graph.  HB_EINVAL outside those ranges. */
int hb_plan_set_config(hb_plan *plan, int waves_per_cu, int msgs_per_lane, int variant);

/* Average duration in milliseconds of the persistent hashing kernel over the runs since
 * the last call, measured with HIP events around it on the plan's stream; -1 if none. */
double hb_plan_kernel_ms(hb_plan *plan);

void hb_plan_destroy(hb_plan *plan);

/*
 * hash_batch_bucketed_noalloc -- for callers that cannot allocate (code under hipGraph
 * capture, serving loops and harnesses that forbid hipMalloc): the batched form of
 * hb_plan_run without a plan.  Same arguments, digests and steps as hb_plan_run with
 * HB_PLAN_LONG_INLINE (bucketing, longest-first persistent launch, long chains beside the
 * bulk in one launch), except that every long chain is a direct chain (no schedule
 * scratch) and nothing is captured in a graph.  The workspace is a static device array of
 * about 4.6 MiB that each GPU the library runs on holds until the process ends; the first
 * call on a device looks up its address there.  No call allocates or frees memory.
 *   n            at most 2^20 messages: larger n returns HB_EINVAL before anything is
 *                enqueued
 * Every call on a GPU uses that GPU's one array (each run clears what it needs first), so
 * calls that overlap on one GPU -- on different streams or from different threads --
 * race and give wrong digests: serialise them, for example on one stream.
 */
int hash_batch_bucketed_noalloc(const uint8_t *algos, int algo, const uint8_t *messages,
                                const uint64_t *offsets, const uint64_t *lengths, uint64_t n,
                                uint8_t *digests_out, void *stream);

/* ------------------------------------------------------------------------------------ */
/* Host-resident inputs: chunked H2D copies overlapped with hashing.                      */
/* ------------------------------------------------------------------------------------ */

/*
 * hash_batch_host -- hash messages that live in host memory.  The messages are split into
 * chunks of about chunk_bytes; chunk k+1 is copied into the device on a copy stream
 * (through pinned staging) while chunk k is hashed on the compute stream, each hash
 * launch gated by an event on its copy.  Digests are copied back to digests_out_host.
 *   algos_host      host, n x uint8 per-message ids, or NULL to use algo
 *   messages_host   host bytes; offsets_host/lengths_host host uint64 arrays
 *   digests_out_host host, n slots (stride 32 with algos_host, else digest size)
 * A batch of at most 16 MiB of payload and at most 2^20 messages is instead hashed where
 * it lies after packing: one plain launch reads the pinned staging buffer through its
 * device mapping and writes the digests to pinned memory, with no copy-engine transfer
 * (HB_HOST_ZERO_COPY_MAX, in bytes, overrides the payload limit; 0 turns this off).
 * Blocking: returns when every digest is in digests_out_host.  Allocates device and
 * pinned buffers and its plans on first use and keeps them for later calls (per thread;
 * a batch holding messages of HB_LONG_MIN_BLOCKS blocks or more adds a plan with the
 * long-chain path and its scratch); its streams are released at the end of each call.
 */
int hash_batch_host(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                    const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                    uint8_t *digests_out_host, uint64_t chunk_bytes);

/*
 * hash_batch_host_split -- the CPU + GPU split of Sec. V-D (Eq. 1-3): host cores hash the
 * trailing messages that hold about cpu_fraction of the payload bytes while the GPU path
 * of hash_batch_host hashes the others, at the same time; the call returns when both
 * halves are in digests_out_host.  Sec. V-D picks the fraction x that balances
 * T_cpu = N P_cpu x / N_core against T_gpu = (P_gpu / N_thread + T_alloc + T_memcpy) N (1 - x)
 * + O_gpu; the caller passes it (hb_cpu_hash_batch measures a host rate for that).
 *   cpu_fraction  in [0, 1]: 0 is hash_batch_host, 1 hashes everything on the host
 *   cpu_threads   host threads for the CPU share (<= 0: all hardware threads)
 * Other arguments and errors as hash_batch_host; HB_EINVAL for a fraction outside [0, 1].
 * The host share is computed by host code of this library (not the GPU kernels), from the
 * same standards, into the same digest layout.
 */
int hash_batch_host_split(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                          const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                          uint8_t *digests_out_host, uint64_t chunk_bytes, double cpu_fraction,
                          int cpu_threads);

/*
 * hb_cpu_hash_batch -- the host-core hashing of hash_batch_host_split on its own: n
 * messages in host memory on `threads` host threads (<= 0: all), digests in the layout of
 * hash_batch_host (stride 32 with algos_host, else the digest size).  Gives the per-byte
 * host cost P_cpu / N_core of Eq. 1.  Blocking; HB_EINVAL for an unknown algorithm or null
 * pointers.
 */
int hb_cpu_hash_batch(const uint8_t *algos_host, int algo, const uint8_t *messages_host,
                      const uint64_t *offsets_host, const uint64_t *lengths_host, uint64_t n,
                      uint8_t *digests_out_host, int threads);

/* ------------------------------------------------------------------------------------ */
/* Serving: continuous batching of hash requests under an HBM budget.                    */
/* ------------------------------------------------------------------------------------ */

typedef struct hb_server hb_server;

/*
 * hb_server_create -- start a serving loop on `device` with a device-memory budget of
 * hbm_budget_bytes (request payload resident at once) and at most max_slots requests in
 * flight.  A background host thread admits queued requests in arrival order while both
 * limits hold; staging threads pack each admitted request's bytes into pinned memory and
 * copy them into the device on a copy stream; staged requests are batched into hashing
 * steps, requests holding a long chain apart from the rest, each kind on its own compute
 * stream, long-chain steps with the plan's long-chain path in one launch: three streams
 * in all (four with two long-chain streams), since streams beyond the process's hardware
 * queues share them and wait behind each other's kernels.  Environment: HB_SERVER_STAGERS
 * staging
 * threads (default 4); HB_SERVER_LONG_STREAMS long-chain streams (default 1, or 2 when
 * the process was started with GPU_MAX_HW_QUEUES >= 8: more long-chain streams only help
 * with more hardware queues than HIP's default four); HB_SERVER_LONG_PLAN_FLAGS the
 * long-chain steps' plan flags (default HB_PLAN_LONG_INLINE: the long-chain path of
 * hb_plan_create in one launch; 0: with a side stream; HB_PLAN_NO_LONG: none);
 * HB_SERVER_COPY_STREAMS copy streams (default 1, or 2 with GPU_MAX_HW_QUEUES >= 8; one
 * copy stream carries about 20-25 GB/s of payload, so a serving process is best started with
 * GPU_MAX_HW_QUEUES=8); HB_SERVER_COPY=kernel copies payload by kernel from the rings'
 * device mapping, not the copy engine.  A request arriving while others run starts as soon
 * as memory and a slot free up, and its work overlaps theirs on the device.
 * HB_SERVER_MODE=resident replaces the steps with one resident serving kernel that requests
 * join while it runs: as soon as a request's payload has landed, its work items (up to 64
 * messages of one algorithm, ordered by algorithm and block count) go into a ring in
 * pinned host memory; the kernel's first wave copies them into device memory and its other
 * waves claim them (several at once when a backlog has built up, while their longest
 * messages sum to at most 64 blocks), hash them -- items of up to 4 long messages, which the
 * loop forms from each algorithm's longest messages while few items are outstanding
 * (HB_SERVER_RESIDENT_LATENCY_ITEMS, default twice the launch's waves), with the whole wave on
 * each chain -- and write the digests and a done flag straight to pinned host memory.  The kernel leaves after 5 ms
 * without items (HB_SERVER_RESIDENT_IDLE_MS) or when the server is destroyed, and the loop
 * starts it again when items wait; one workgroup per two CUs (HB_SERVER_RESIDENT_WGS sets the
 * count: with one on every CU the payload copies, kernels themselves, lag at high load).  While it
 * runs, device-wide synchronisations of the process (hipDeviceSynchronize, hipFree) wait
 * for it.  Returns HB_EINVAL for a null server pointer,
 * a budget below 256 bytes or max_slots <= 0, HB_ENOMEM if the device arena or pinned
 * buffers cannot be allocated, HB_EHIP for other runtime failures.
 */
int hb_server_create(hb_server **server, int device, uint64_t hbm_budget_bytes, int max_slots);

/*
 * hb_server_submit -- queue one request (host pointers, valid until completion).
 *   algo_or_mixed  an algorithm id, or -1 to use algos[] per message
 *   algos          host n x uint8 ids when algo_or_mixed == -1, else ignored
 *   digests_out    host, n slots (stride 32 when mixed, else digest size)
 * Returns HB_EINVAL for malformed requests and HB_EBUDGET for a request that could never
 * fit the budget; either fails alone.  On success *ticket identifies the request.
 */
int hb_server_submit(hb_server *server, int algo_or_mixed, const uint8_t *algos,
                     const uint8_t *messages, const uint64_t *offsets, const uint64_t *lengths,
                     uint64_t n, uint8_t *digests_out, uint64_t *ticket);

/* Non-blocking completion check: *done = 1 when finished, with its status in *status.  For
 * a finished request that failed, hb_last_error() on the calling thread then returns the
 * failure's explanation, whichever server thread raised it. */
int hb_server_poll(hb_server *server, uint64_t ticket, int *done, int *status);

/* Cancel a request that has not been admitted yet: it leaves the queue and finishes with
 * status HB_ECANCELED (its digest slots untouched).  HB_EBUSY once it has been admitted
 * (it then runs to completion), HB_EINVAL for an unknown ticket. */
int hb_server_cancel(hb_server *server, uint64_t ticket);

/* Drop the record of a finished request (after its status, times or trace have been
 * read); the ticket is unknown afterwards.  A server keeps every request's record until
 * this call or hb_server_destroy.  HB_EBUSY if the request has not finished. */
int hb_server_release(hb_server *server, uint64_t ticket);

/* Block until the request completes (or timeout_ms elapses, -1 = forever: HB_EBUSY on
 * timeout); *status receives its status.  If the request failed, hb_last_error() on the
 * calling thread returns the failure's explanation, whichever server thread raised it. */
int hb_server_wait(hb_server *server, uint64_t ticket, int64_t timeout_ms, int *status);

/* Per-request timestamps in seconds on the server's steady clock: arrival (submit),
 * admission, input resident on the device, digests ready on the host. */
int hb_server_times(hb_server *server, uint64_t ticket, double *t_submit, double *t_admit,
                    double *t_h2d_done, double *t_done);

/* Per-request trace, for locating where a request's latency goes.  Fills t[0..nt) with
 * times in seconds on the server's steady clock, in the order of the HB_TRACE_* indices
 * (entries past HB_TRACE_COUNT are set to 0):
 *   SUBMIT       hb_server_submit returned the ticket
 *   ADMIT        admitted (arena range and slot reserved)
 *   STAGE_BEGIN  a staging thread started packing it into pinned memory
 *   STAGE_END    its last host-to-device copy was enqueued
 *   H2D_DONE     that copy completed
 *   LAUNCH       the device step holding it was enqueued (possibly before H2D_DONE: the
 *                step then waits on the device for the copy)
 *   EXEC_BEGIN   that step's inputs and metadata were resident and hashing could start
 *   EXEC_END     that step's digests were back in pinned host memory
 *   DONE         its digests were in the caller's buffer and it was marked done
 * H2D_DONE, EXEC_BEGIN and EXEC_END are the times the serving loop saw the device events
 * complete (late by at most one pass of its polling loop), so every entry is on the same
 * host clock and SUBMIT <= ADMIT <= STAGE_BEGIN <= STAGE_END <= H2D_DONE <= EXEC_BEGIN <=
 * EXEC_END <= DONE, LAUNCH <= EXEC_BEGIN.  Times not reached yet are 0.  Returns HB_EINVAL
 * for a null server, a negative nt, a null t with nt > 0, or an unknown ticket. */
enum {
    HB_TRACE_SUBMIT = 0,
    HB_TRACE_ADMIT = 1,
    HB_TRACE_STAGE_BEGIN = 2,
    HB_TRACE_STAGE_END = 3,
    HB_TRACE_H2D_DONE = 4,
    HB_TRACE_LAUNCH = 5,
    HB_TRACE_EXEC_BEGIN = 6,
    HB_TRACE_EXEC_END = 7,
    HB_TRACE_DONE = 8,
    HB_TRACE_COUNT = 9
};
int hb_server_trace(hb_server *server, uint64_t ticket, double *t, int nt);

/* Counters: requests completed, device steps launched, admission stalls (a queued head
 * request held back by the budget or slot limit), peak resident bytes. */
int hb_server_stats(hb_server *server, uint64_t *completed, uint64_t *steps, uint64_t *stalls,
                    uint64_t *peak_bytes);

/* Current time on the server clock (seconds), for timestamps taken by the caller. */
double hb_server_now(hb_server *server);

/* Drain outstanding requests and stop the loop. */
void hb_server_destroy(hb_server *server);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
