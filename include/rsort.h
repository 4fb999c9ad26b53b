/*
 * rsort -- robust sample sort for AMD MI355X (gfx950).
 *
 * C ABI of librsort.so.  Every data pointer is a DEVICE pointer owned by the
 * caller unless stated otherwise; `stream` is a hipStream_t passed as void*
 * (NULL = the null stream).  Calls return an int status (RSORT_OK = 0, or a
 * negative error code); no exception crosses the ABI.
 *
 * Problem statement (paper, Section 2 "Preliminaries"): n input elements are
 * to be output globally sorted.  Following the paper's robustness scheme
 * (Section 5; Appendix F for the work-inefficient sort, Appendix G for the
 * multi-level sample sort) keys are made unique by their input position, so
 * the output is the unique permutation pi of 0..n-1 with
 * (ord(x[pi(r)]), pi(r)) strictly increasing in r: ascending keys, equal keys
 * in ascending input position.  ord is the identity for unsigned keys and the
 * IEEE 754 totalOrder map for f32 keys (-NaN < -inf < ... < -0 < +0 < ... <
 * +inf < +NaN; -0 and +0 are different keys).  Output keys keep their
 * original bits.
 *
 * Asynchrony: rsort_plain and rsort_segmented enqueue work on `stream` and
 * return without synchronising the host.  Argument errors detectable on the
 * host are returned immediately; errors only detectable on the device (e.g.
 * decreasing segment offsets) are recorded in the workspace status word and
 * read back with rsort_workspace_status().
 */
#ifndef RSORT_H
#define RSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { RSORT_U32 = 0, RSORT_U64 = 1, RSORT_F32 = 2 } rsort_key_t;

enum {
  RSORT_OK = 0,
  RSORT_PENDING = 1,
  RSORT_EINVAL = -1,   /* bad argument */
  RSORT_ENOMEM = -2,   /* workspace too small / request larger than a budget */
  RSORT_EDEVICE = -3,  /* HIP runtime or device error */
  RSORT_EBUSY = -4,    /* server queue full */
  RSORT_ENOTFOUND = -5 /* unknown ticket */
};

/* Static string for a status code. */
const char *rsort_strerror(int code);

/* ABI version (major * 100 + minor). */
int rsort_version(void);

/* ------------------------------------------------------------------------
 * Plain sort (multilevel sample sort, paper Appendix G; single level for
 * small n, plain LDS sort when n fits one workgroup).
 *
 * rsort_plain_workspace: bytes of device workspace rsort_plain needs for n
 * keys of type kt (0 if kt is invalid).
 *
 * rsort_plain: sorts keys_in[0..n) into keys_out[0..n) and, if perm_out is
 * not NULL, writes perm_out[r] = pi(r) (u32 input positions).
 *   kt          key type; keys_in/keys_out hold 4-byte (u32, f32) or 8-byte
 *               (u64) elements, contiguous.
 *   n           0 <= n < 2^32 - 1; n == 0 is a no-op.
 *   keys_out    must not overlap keys_in (out-of-place only).
 *   workspace   device memory of at least rsort_plain_workspace(kt, n) bytes,
 *               used only for the duration of the enqueued work.
 * Errors: RSORT_EINVAL for a NULL pointer with n > 0, unknown kt, n too
 * large, or overlapping buffers; RSORT_ENOMEM if workspace_bytes is too
 * small; RSORT_EDEVICE if a launch fails.
 * ---------------------------------------------------------------------- */
size_t rsort_plain_workspace(rsort_key_t kt, uint64_t n);
int rsort_plain(rsort_key_t kt, const void *keys_in, uint64_t n, void *keys_out, uint32_t *perm_out,
                void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Plain sort with 64-bit positions, for arrays of 2^32 - 1 keys or more
 * (n <= 2^36).  Same definition as rsort_plain with positions 0..n-1 as
 * u64: perm_out (NULL = keys only) is a device u64 [n].
 * One top level of the multilevel sample sort (Appendix G) splits the keys
 * into 256 buckets by (key, 64-bit position) splitters with a stable scatter
 * (each bucket keeps input order), then every bucket is sorted with 32-bit
 * bucket-local positions -- which order equal keys as the global positions
 * do -- and the permutation is gathered back to global positions.  Works for
 * any n >= 0; below 2^32 - 1 keys rsort_plain is faster.
 *   workspace  rsort_plain64_workspace(kt, n) bytes (about 34 B per u32 /
 *              f32 key and 46 B per u64 key); its status word
 *              (rsort_workspace_status) becomes RSORT_EINVAL if a bucket
 *              reached 2^32 - 1 keys (keys too skewed for 256 buckets).
 * Stream-ordered and asynchronous.  Errors: RSORT_EINVAL (kt, n > 2^36,
 * NULL pointers with n > 0, overlapping buffers), RSORT_ENOMEM (workspace
 * too small), RSORT_EDEVICE.
 * ---------------------------------------------------------------------- */
size_t rsort_plain64_workspace(rsort_key_t kt, uint64_t n);
int rsort_plain64(rsort_key_t kt, const void *keys_in, uint64_t n, void *keys_out, uint64_t *perm_out,
                  void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * rsort_plain without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, hosts that
 * forbid allocation while running).  Same sort, arguments and output as
 * rsort_plain; the scratch is a 64 MiB device array that the library holds
 * statically, one per GPU it runs on, until the process ends.  Nothing is
 * allocated by the call.
 *   n  must need at most 64 MiB of workspace, i.e.
 *      rsort_plain_workspace(kt, n) <= 64 MiB: with the default tuning up to
 *      about 2.5 million u64 keys or 3.1 million u32 / f32 keys; larger n
 *      returns RSORT_ENOMEM before any device call.
 * Calls on one GPU share its scratch array (each call resets what it uses):
 * calls whose work overlaps on the same GPU (e.g. on two streams) race and
 * must be ordered by the caller.
 * Errors: as rsort_plain; RSORT_ENOMEM for n beyond the scratch;
 * RSORT_EDEVICE if the scratch address cannot be obtained.
 * ---------------------------------------------------------------------- */
int rsort_plain_noalloc(rsort_key_t kt, const void *keys_in, uint64_t n, void *keys_out, uint32_t *perm_out,
                        void *stream);

/* ------------------------------------------------------------------------
 * Robust hypercube quicksort with workgroups as PEs (paper Section 6,
 * Algorithm 2) for one array, its exchanges going through HBM.  Sorts by the
 * definition above (u32 or f32 keys only).
 *
 * p = 2^log2_p PEs (1 <= log2_p <= 8), each holding a packed part of the
 * array.  Steps:
 *   1. random redistribution (Section 3.1): in each of log2_p rounds every PE
 *      keeps one random half of its part and sends the other half to its
 *      partner across one cube dimension;
 *   2. every PE sorts its part in LDS (at most 8192 keys: ceil(n / p) must
 *      not exceed 8192);
 *   3. for each dimension, highest first, the binary-tree median (Section
 *      3.2, even window k, 2 <= k <= 16) of each subcube is its splitter;
 *      PEs split their parts at it and exchange and merge halves.
 * tie_break selects how a PE splits its sorted part at the splitter s:
 *   1  by (key, position), as the robust sample sort orders elements: the
 *      output is the definition above;
 *   0  by key only (ablation without tie-breaking): the same output, only
 *      the load balance differs (equal keys pile up on one side);
 *   2  the paper's local scheme (Section 6): of the m copies of s's key in a
 *      part a = a_l s^m a_r, keep x in L = a_l s^x with |L| closest to
 *      |a| / 2.  keys_out is the sorted key sequence, but equal keys may
 *      appear in any order, so perm_out is one valid sorting permutation,
 *      not necessarily the one defined above.
 * seed drives the shuffle and the median's coins.
 *
 *   keys_in   device u32/f32 [n]; keys_out device [n]; perm_out device u32
 *             [n] or NULL.
 *   load_out  device u32 [log2_p + 1] or NULL: the largest PE part after the
 *             redistribution, then after each exchange round.
 *   workspace rsort_rquick_mw_workspace(n, log2_p) bytes (0 = shape not
 *             supported).
 * Stream-ordered and asynchronous.  A device-side guard sets the workspace
 * status (rsort_workspace_status) to RSORT_EINVAL if a PE part ever exceeds
 * 8192 keys before its LDS sort; the shuffle keeps every part within one key
 * of ceil(n / p), so accepted shapes leave it at RSORT_OK.
 * Errors: RSORT_EINVAL (key type, n >=
 * 2^32 - 1, log2_p, k, tie_break, ceil(n / p) > 8192, NULL pointers with n > 0,
 * overlapping buffers), RSORT_ENOMEM (workspace too small), RSORT_EDEVICE.
 * ---------------------------------------------------------------------- */
size_t rsort_rquick_mw_workspace(uint64_t n, uint32_t log2_p);
int rsort_rquick_mw(rsort_key_t kt, const void *keys_in, uint64_t n, uint32_t log2_p, uint32_t k, int tie_break,
                    uint64_t seed, void *keys_out, uint32_t *perm_out, uint32_t *load_out, void *workspace,
                    size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Segmented (batched) sort: num_segs independent arrays in one call, each
 * sorted by the same definition with SEGMENT-LOCAL positions.  The work is a
 * fixed sequence of launches independent of num_segs; each segment is routed
 * to an algorithm by its size class (the paper's observation that different
 * algorithms win at different input sizes, Section 4 and Section 7): the
 * all-pairs rank sort RFIS (Section 5), robust quicksort RQuick (Section 6),
 * an LDS merge sort, or multilevel sample-sort levels followed by the LDS
 * sort of the final buckets.
 *
 *   seg_offsets  device array of num_segs + 1 u64: seg_offsets[0] = 0,
 *                nondecreasing, seg_offsets[num_segs] = n_total; segment s
 *                is [seg_offsets[s], seg_offsets[s+1]).  Segments must be
 *                shorter than 2^32 - 1.  A decreasing offset sets the
 *                workspace status to RSORT_EINVAL and leaves outputs undefined.
 *   payload_in   optional (NULL) u32 values carried with the keys:
 *                payload_out[r] = payload_in[start + pi_s(r - start)].
 *   perm_out     optional (NULL): segment-local positions pi_s.
 * Errors as for rsort_plain.
 * ---------------------------------------------------------------------- */
size_t rsort_segmented_workspace(rsort_key_t kt, uint64_t n_total, uint32_t num_segs,
                                 int has_payload);
int rsort_segmented(rsort_key_t kt, const void *keys_in, const uint32_t *payload_in,
                    const uint64_t *seg_offsets, uint32_t num_segs, uint64_t n_total,
                    void *keys_out, uint32_t *payload_out, uint32_t *perm_out, void *workspace,
                    size_t workspace_bytes, void *stream);

/* Status word of a workspace after the work enqueued on `stream` has
 * completed (synchronises `stream`).  Returns RSORT_OK or the device-detected
 * error. */
int rsort_workspace_status(const void *workspace, void *stream);

/* ------------------------------------------------------------------------
 * Diagnostics of the last call that used `workspace` (synchronises stream).
 * Level 0 of segment 0 is recorded: its splitters in sorted order (the
 * sample elements chosen, as (ord key, position) pairs; keys are u64 holding
 * the ordinal key -- for f32 keys the totalOrder bits) and the sizes of its
 * buckets.  Host output arrays:
 *   spl_keys[511], spl_pos[511], bucket_sizes[512]; *num_buckets receives the
 *   bucket count k (0 if no split happened), *levels the number of levels
 *   enqueued, level_max[8] the largest bucket produced per level and
 *   level_buckets[8] the number of non-empty buckets per level, *oversize the
 *   number of final buckets that needed the fallback sort.
 * ---------------------------------------------------------------------- */
int rsort_stats(const void *workspace, void *stream, uint64_t *spl_keys, uint32_t *spl_pos,
                uint32_t *bucket_sizes, uint32_t *num_buckets, uint32_t *levels,
                uint32_t *level_max, uint32_t *level_buckets, uint32_t *oversize);

/* Size classes of the final buckets of the last call that used `workspace`
 * (synchronises stream).  For up to max_classes classes: the largest bucket
 * the class sorts (0xFFFFFFFF for the global-memory fallback class), the
 * number of buckets and the number of keys routed to it.  Any output may be
 * NULL.  Returns the number of classes (>= 0) or an error. */
int rsort_class_stats(const void *workspace, void *stream, uint32_t max_classes,
                      uint32_t *class_max, uint32_t *buckets, uint64_t *keys);

/* ------------------------------------------------------------------------
 * Tuning.  Fields set to 0 keep their current value.  Applies to calls made
 * after it returns (process-wide, not thread-safe against concurrent calls).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t oversample;   /* samples per bucket a (sample size a * k; default 32) */
  uint32_t target;       /* bucket size a level aims for (default 6144, at most cap / 2) */
  uint32_t cap;          /* largest bucket sorted in LDS; larger ones are split */
  uint32_t max_levels;   /* upper bound on sample-sort levels */
  uint32_t rfis_max;     /* segments <= rfis_max use RFIS (default 64; 0 keeps, 1 disables) */
  uint32_t rquick_max;   /* segments <= rquick_max (and > rfis_max) use RQuick */
  uint64_t seed;         /* seed of the sample positions and coin flips */
  uint32_t tile_log2;    /* log2 of keys per scatter tile (12 or 13; counting uses 12) */
  uint32_t force_fallback; /* debug: 1 = every final bucket > 64 takes the
                              global-memory fallback sort, 2 = off (0 keeps) */
  uint32_t extra_levels;   /* levels beyond the fewest that reach the target
                              bucket size (at most 4): more, smaller levels
                              shorten nothing but lengthen each scatter's runs;
                              the value is stored plus one (1 = none, 0 keeps) */
  uint32_t class_shape;    /* bit c set: final-size class c (0..8) runs its word
                              sort with the alternative workgroup shape (twice
                              the threads, half the keys per thread) -- bit 31
                              must be set for the mask to be taken (0 keeps) */
} rsort_tuning;

int rsort_get_tuning(rsort_tuning *out);
int rsort_set_tuning(const rsort_tuning *in);

/* ------------------------------------------------------------------------
 * Sort server (continuous batching).  At creation the server reserves
 * hbm_budget_bytes of device memory as its scratch arena and creates
 * max_inflight HIP streams (slots).  Every in-flight sort takes its scratch
 * (workspace, and for packed batches the packed buffers) from the arena and
 * returns it on completion; no device memory is allocated while serving.
 *
 * Requests of more than 2^20 keys are admitted in arrival order, one per
 * slot, when their scratch fits the arena.  Smaller requests are queued and
 * packed: whenever a small-request slot is free (at most two batches in
 * flight), the queued small requests of the oldest one's key type (up to 1024
 * requests and 2^24 keys, within the arena's largest free block) are sorted
 * by one segmented sort between one gather and one scatter-back launch.  A
 * request's result is bit-identical to the one it gets alone.  A device
 * error in a packed batch is reported to every request of that batch.
 *
 * Request buffers are device pointers owned by the caller and must stay
 * valid until rsort_poll returns something other than RSORT_PENDING.  The
 * server's streams do not wait on any stream of the caller: keys_in must
 * already hold its final contents on the device when rsort_submit is called
 * (e.g. the producing stream has been synchronised), and keys_out / perm_out
 * must not be read or written by other work until the ticket has finished.
 * Setting the environment variable RSORT_SERVER_LOG to a file path makes
 * each server append one line per launch (slot, requests, keys, host
 * enqueue time) and per completion to that file.
 * ---------------------------------------------------------------------- */
typedef struct rsort_server rsort_server;

typedef struct {
  rsort_key_t kt;
  const void *keys_in;
  uint64_t n;
  void *keys_out;
  uint32_t *perm_out; /* may be NULL */
} rsort_request;

typedef struct {
  int status;         /* RSORT_OK, RSORT_PENDING or an error */
  uint64_t t_submit_ns; /* CLOCK_MONOTONIC timestamps */
  uint64_t t_start_ns;  /* admitted and enqueued */
  uint64_t t_done_ns;   /* completion observed by the server */
  uint32_t batch_size;  /* requests sorted in the same launch */
  uint64_t dev_begin_ns; /* device timestamps of the start and the end of the */
  uint64_t dev_end_ns;   /* launch sequence that sorted the request, in ns after an
                            event the server records at creation (0 for the fake
                            executor or on error); requests whose [begin, end)
                            intervals intersect were in flight on the device at
                            the same time */
} rsort_result;

/* Arena bytes one request of n keys takes when it runs alone (0 for n == 0
 * or a bad key type).  Requests above hbm_budget_bytes get RSORT_ENOMEM. */
size_t rsort_server_request_bytes(rsort_key_t kt, uint64_t n);
/* device: HIP device ordinal, or < 0 for a host-only fake executor (tests of
 * the scheduling logic: no GPU, buffers untouched).  max_inflight: slots
 * (1..64); with two or more, slot 0 serves only requests of at most 2^20 keys.
 * RSORT_ENOMEM if the arena cannot be allocated. */
int rsort_server_create(int device, uint64_t hbm_budget_bytes, uint32_t max_inflight,
                        rsort_server **out);
/* Waits for every admitted request, then frees server memory. */
int rsort_server_destroy(rsort_server *s);
/* Non-blocking.  RSORT_ENOMEM if the request alone exceeds the budget,
 * RSORT_EINVAL for bad fields.  *ticket_out receives a unique ticket. */
int rsort_submit(rsort_server *s, const rsort_request *r, uint64_t *ticket_out);
/* RSORT_PENDING while queued or running; otherwise the request's final
 * status, with timestamps in *out (may be NULL).  A finished ticket stays
 * queryable until rsort_release. RSORT_ENOTFOUND for unknown tickets. */
int rsort_poll(rsort_server *s, uint64_t ticket, rsort_result *out);
/* Blocks until the ticket finishes (or timeout_ms elapses: RSORT_PENDING). */
int rsort_wait(rsort_server *s, uint64_t ticket, uint32_t timeout_ms, rsort_result *out);
/* Forget a finished ticket. */
int rsort_release(rsort_server *s, uint64_t ticket);
/* Counters: requests queued, running, finished; arena bytes in use. */
int rsort_server_counters(rsort_server *s, uint64_t *queued, uint64_t *running,
                          uint64_t *finished, uint64_t *bytes_in_use);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support, process-wide).  rsort_timing_begin()
 * starts bracketing every kernel this library launches with HIP events on
 * the launch's own stream.  rsort_timing_end() stops, synchronises the device
 * and reports per kernel name (up to max_entries, names truncated to
 * name_len - 1 characters in the caller's char[max_entries][name_len]) the
 * number of launches and their summed duration in milliseconds.
 * ---------------------------------------------------------------------- */
int rsort_timing_begin(void);
int rsort_timing_end(uint32_t max_entries, char *names, uint32_t name_len, uint32_t *launches,
                     double *total_ms, uint32_t *n_entries);

/* ------------------------------------------------------------------------
 * Bandwidth probe (measurement support): kind 0 reads bytes of src once
 * (16 bytes per lane per access) and writes one 32-bit word per workgroup to
 * dst (at most 8 words per compute unit, so dst needs 8 * CUs * 4 bytes);
 * kind 1 copies bytes of src to dst.  bytes and both pointers must be
 * multiples of 16.  Stream-ordered; the rates these two reach are the
 * practical ceilings of a read-only and of a read + write pass.
 * Errors: RSORT_EINVAL (kind, alignment, NULL), RSORT_EDEVICE.
 * ---------------------------------------------------------------------- */
int rsort_bandwidth_probe(int kind, const void *src, void *dst, uint64_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * Binary-tree approximate median (paper Section 3.2), computed on the device
 * for num_problems independent problems of p = 2^log2_p leaves each.
 *   vals      device u64 values of all problems back to back (unique within a
 *             problem); problem q's leaf l holds
 *             vals[q*per_problem + leaf_off[q*(p+1) + l] .. + leaf_off[q*(p+1) + l + 1]).
 *             A leaf holds at most 64 values, not necessarily sorted.
 *   leaf_off  device u64 [num_problems * (p + 1)], nondecreasing per problem.
 *   coins     device u8 [num_problems * (p + 1)]: p leaf coins (used by leaves
 *             with an odd count: 0 = lower middle, 1 = upper middle), then the
 *             root coin (0 = element k/2, 1 = element k/2 + 1 of the root window).
 *   k         even window size, 2 <= k <= 32.
 *   out       device u64 [2 * num_problems]: {value, side} per problem, side
 *             = 0 for a real value, 1 for the below-all sentinel, 2 for the
 *             above-all sentinel (value 0 then).
 * Leaves forward the k values around their median, padded with the two
 * sentinels; inner nodes merge their children's windows and forward the
 * middle k; the root returns one of its two middle values.
 * workspace: rsort_median_tree_workspace(log2_p, k, num_problems) bytes.
 * Errors: RSORT_EINVAL (k odd / out of range, log2_p > 24, NULL pointers),
 * RSORT_ENOMEM (workspace too small), RSORT_EDEVICE.
 * ---------------------------------------------------------------------- */
size_t rsort_median_tree_workspace(uint32_t log2_p, uint32_t k, uint32_t num_problems);
int rsort_median_tree(const uint64_t *vals, uint64_t per_problem, const uint64_t *leaf_off,
                      uint32_t log2_p, uint32_t k, const uint8_t *coins, uint32_t num_problems,
                      uint64_t *out, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RSORT_H */
