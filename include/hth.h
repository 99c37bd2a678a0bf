/*
 * libhth: HalftimeHash on AMD Instinct MI355X (gfx950).
 *
 * The hash family H(s, x) of the paper (§1: a map from a seed s and a byte
 * string x to a 16, 24, 32 or 40 byte value, almost universal among strings
 * of equal length, §2) computed by hand-written HIP kernels.  Every result is
 * bit-for-bit the value the family defines; there is no approximate mode.
 *
 * Family (paper §5.1, §6.1): b = 8 64-bit words per block, code symbols of
 * w = 3 words, tree fanout f = 8; per width (d, e, k) = (6,7,2), (7,9,3),
 * (7,10,4), (5,9,5); the k x e combine matrices printed in §5.1; systematic
 * GF(8) MDS erasure codes of distance k; k trees of NH-variant nodes (§3.2)
 * over the EHC outputs with the stack construction of Eq. (3) in base 8;
 * one final NH per tree (§5.2); the tail hashed k times with Toeplitz keys
 * (§6.1); an NH of the byte length added to every output word (§2 asks for
 * the length to be appended so that different lengths also separate).
 *
 * Conventions of every call:
 *   - Return value: HTH_OK (0) or a negative hth_status.  On error nothing
 *     is enqueued and no output is written; hth_last_error() gives a
 *     message (thread-local, valid until the next call on the thread).
 *   - "device pointer": memory of the current HIP device (hipMalloc, torch
 *     CUDA tensors).  "host pointer": ordinary process memory.
 *   - Calls that take a stream enqueue work on it and return without
 *     waiting; inputs must stay valid and unmodified, and outputs must not
 *     be read, until that work is complete.  Stream 0 is the null stream.
 *   - All calls are thread-safe.  Two hth_hash_batch calls in flight on
 *     different streams use different scratch areas and may overlap.
 */
#ifndef HTH_H
#define HTH_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hth_status;
#define HTH_OK 0
#define HTH_E_INVALID (-1)   /* bad argument (null pointer, unsupported width, ...) */
#define HTH_E_OOM (-2)       /* device or host allocation failed */
#define HTH_E_HIP (-3)       /* a HIP runtime call failed */
#define HTH_E_BUSY (-4)      /* not ready yet / admission deferred */
#define HTH_E_TOO_LARGE (-5) /* request exceeds a configured limit */

/* Thread-local description of the last failure on this thread. */
const char *hth_last_error(void);

/* Number of 64-bit entropy words of a seed (all four widths together). */
size_t hth_entropy_words(void);

/* ------------------------------------------------------------------------ */
/* Seeds.  The family is parameterised by random entropy words (the paper's */
/* "input entropy", §2, §6.2).  A seed object holds them in device memory,  */
/* is immutable after creation and may be shared by any number of streams.  */
/* ------------------------------------------------------------------------ */

typedef struct hth_seed hth_seed;

/* Fill the entropy of all widths from a 64-bit user seed: word i is output i
   of splitmix64 started at state user_seed (Steele, Lea and Flood 2014).
   The host computes the words and copies them to the device on `stream`.
   *out is owned by the caller until hth_seed_free.
   Errors: HTH_E_INVALID (out null), HTH_E_OOM, HTH_E_HIP. */
hth_status hth_expand_seed(uint64_t user_seed, hth_seed **out, hipStream_t stream);

/* Same, from caller-provided raw entropy: `words` is a host pointer to
   n_words = hth_entropy_words() words (layout: for each width 16, 24, 32, 40
   in turn, [EHC keys e*w][tree keys k*20*7][final keys k*20*7*8]
   [tail keys 8*d*w + k - 1][length keys k]).  The words are copied; the
   caller keeps ownership of `words`.
   Errors: HTH_E_INVALID (null pointer or wrong n_words), HTH_E_OOM, HTH_E_HIP. */
hth_status hth_seed_from_entropy(const uint64_t *words, size_t n_words, hth_seed **out,
                                 hipStream_t stream);

/* The 256-bit block family.  §6.3 makes the block size b (64-bit words per
   block) the machine's vector width, and each b its own family: b = 8 (the
   default, used by the calls above) or b = 4, the paper's 256-bit variant.
   With b = 4 an EHC execution is 32*d*w bytes (576 / 672 / 672 / 480 for
   the widths 16 / 24 / 32 / 40), there are 4 instances, and the layout per
   width is [EHC e*w][tree k*20*7][final k*20*7*4][tail 4*d*w + k - 1][len k].
   A seed carries its b; hth_hash_batch, captured batches and servers hash
   with the family of the seed they are given.  block_words must be 4 or 8
   (HTH_E_INVALID otherwise); other errors as the b = 8 calls. */
size_t hth_entropy_words_b(uint32_t block_words);
hth_status hth_expand_seed_b(uint64_t user_seed, uint32_t block_words, hth_seed **out, hipStream_t stream);
hth_status hth_seed_from_entropy_b(const uint64_t *words, size_t n_words, uint32_t block_words, hth_seed **out,
                                   hipStream_t stream);
/* Block size of a seed's family (0 for null). */
uint32_t hth_seed_block_words(const hth_seed *seed);

/* Copy a seed's entropy words to host memory (n_words must equal the
   seed's entropy size).  Synchronous. */
hth_status hth_seed_entropy(const hth_seed *seed, uint64_t *host_words, size_t n_words);

/* Release a seed.  Work already enqueued with it must have completed.
   Null is accepted. */
hth_status hth_seed_free(hth_seed *seed);

/* ------------------------------------------------------------------------ */
/* Batched hashing.                                                          */
/* ------------------------------------------------------------------------ */

/* Hash `count` byte strings with one family member H(seed, .): the seeded
 * hash family of §1, almost-universal among strings of equal length (§2),
 * computed as EHC per block (§3.3, §4, §5.1), the tree of Eq. (3) with the
 * final NH (§5.2), the Toeplitz tail (§6.1) and a length term.
 *
 *   bytes    device pointer; string i is bytes[offsets[i], offsets[i] +
 *            lengths[i]).  No alignment is required; strings may overlap.
 *   offsets  device pointer to count uint64_t.
 *   lengths  device pointer to count uint64_t.
 *   out      device pointer to count * out_width bytes; row i receives the
 *            out_width-byte value of string i: k = out_width / 8 words,
 *            little endian, tree 0 first.
 *   out_width  16, 24, 32 or 40.
 *
 * out[i] depends only on the seed and string i, never on the rest of the
 * batch.  The call enqueues a short planning step, one persistent hashing
 * kernel, a small kernel for the strings shorter than one EHC execution
 * (tail only) and one for the strings of 1 .. 7 executions on `stream` and
 * returns.  Scratch memory comes from a per-stream workspace
 * that the library grows on the host as `count` grows (hth_reserve
 * pre-allocates it, e.g. before stream capture: a call inside a capture never
 * allocates and fails with HTH_E_INVALID if the workspace is too small).
 * Batches whose strings total more than about 2^20 * 128 * 8^5 executions
 * (far beyond device memory unless strings overlap) are flagged by the
 * device and produce no output; hth_batch_check reports it.
 * Errors: HTH_E_INVALID (null seed/pointers with count > 0, bad out_width),
 * HTH_E_OOM, HTH_E_HIP.  count == 0 enqueues nothing. */
hth_status hth_hash_batch(const hth_seed *seed, const uint8_t *bytes, const uint64_t *offsets,
                          const uint64_t *lengths, uint64_t count, uint8_t *out, uint32_t out_width,
                          hipStream_t stream);

/* hth_hash_batch, and also record `main_start` and `main_stop` (events the
   caller created with hipEventCreate; either may be null) on `stream`
   immediately before and after the hashing (the persistent kernel and the
   tail-only kernel), so that the caller can time it without the planning
   step, which runs before main_start.
   Same arguments, errors and semantics as hth_hash_batch otherwise. */
hth_status hth_hash_batch_timed(const hth_seed *seed, const uint8_t *bytes, const uint64_t *offsets,
                                const uint64_t *lengths, uint64_t count, uint8_t *out,
                                uint32_t out_width, hipStream_t stream, hipEvent_t main_start,
                                hipEvent_t main_stop);

/* ------------------------------------------------------------------------ */
/* Composition with a short-input family (§1: a universe-collapsing family   */
/* reduces each long string to a few bytes, which a short-input family then  */
/* hashes as if they were the input; §7 names pairing HalftimeHash with a    */
/* fast short-input family as future work).                                  */
/* ------------------------------------------------------------------------ */

/* The short-input family is simple tabulation over c + 1 byte characters,
   c = inner_width (16, 24, 32 or 40), with one table of 256 random 64-bit
   words per character: tables[i * 256 + v] = T_i[v], i = 0 .. c.  The key of
   a string x of L bytes is
     L <= c:  characters 0 .. c-1 = x zero-padded to c bytes, character c = L
              (the string is tabulated directly: no HalftimeHash work);
     L >  c:  characters 0 .. c-1 = the c-byte HalftimeHash value of x
              (hth_hash_batch with out_width c), character c = 255;
   and the 64-bit result is the XOR of T_i[character i] over i = 0 .. c.
   Keys of the two kinds always differ in character c, and simple tabulation
   makes any two distinct keys collide with probability 2^-64, so two
   distinct strings collide with probability at most eps_c + 2^-64 (eps_c of
   the inner width's family, §6.2).

   Words of the tables for inner width c: (c + 1) * 256, 0 for another width. */
size_t hth_tab_words(uint32_t inner_width);

/* Fill host memory `words` (n_words must equal hth_tab_words(inner_width))
   with tables: word i = output i of splitmix64 started at user_seed (the
   generator of hth_expand_seed; pick a user seed independent of the hashing
   seed's).  Errors: HTH_E_INVALID. */
hth_status hth_tab_expand(uint64_t user_seed, uint32_t inner_width, uint64_t *words, size_t n_words);

/* The composed 64-bit hash of `count` strings.  Arguments as hth_hash_batch,
   and:
     tables  device pointer, hth_tab_words(inner_width) words, 8-byte aligned,
             owned by the caller (valid until `stream` reaches this work);
     out     device pointer to count uint64_t, 8-byte aligned.
   Enqueues the planner and hashing kernels of hth_hash_batch for the strings
   longer than 64 bytes (their values go to the stream's workspace), then one
   tabulation kernel for every string, on `stream`; that kernel computes the
   HalftimeHash value of a string of inner_width + 1 .. 64 bytes itself (the
   tail and length terms of a string shorter than one execution).  Same workspace
   rules as hth_hash_batch.  Errors: HTH_E_INVALID (as hth_hash_batch, null
   or misaligned tables/out with count > 0), HTH_E_OOM, HTH_E_HIP. */
hth_status hth_hash_batch64(const hth_seed *seed, const uint64_t *tables, const uint8_t *bytes,
                            const uint64_t *offsets, const uint64_t *lengths, uint64_t count, uint64_t *out,
                            uint32_t inner_width, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Captured batches (HIP graphs).                                            */
/* ------------------------------------------------------------------------ */

typedef struct hth_batch_graph hth_batch_graph;

/* Capture one hth_hash_batch call (planner and hashing kernel) into a HIP
   graph for repeated launches: the pointers and count are fixed at creation,
   the contents of bytes/offsets/lengths may change between launches (every
   launch plans from the device arrays again).  The graph owns a private
   workspace, so launches of one graph must not overlap (launch it on one
   stream, or order the streams); different graphs are independent.  The
   captured work contains kernels only (no memset nodes).  Synchronous
   with respect to the host while it captures.
   Errors: HTH_E_INVALID (as hth_hash_batch, or count == 0), HTH_E_OOM,
   HTH_E_HIP. */
hth_status hth_batch_graph_create(const hth_seed *seed, const uint8_t *bytes, const uint64_t *offsets,
                                  const uint64_t *lengths, uint64_t count, uint8_t *out,
                                  uint32_t out_width, hth_batch_graph **graph);

/* Enqueue one launch of the captured batch on `stream`. */
hth_status hth_batch_graph_launch(hth_batch_graph *graph, hipStream_t stream);

/* Synchronise `stream` and report the planner status of the graph's last
   launch (HTH_OK or HTH_E_TOO_LARGE, as hth_batch_check). */
hth_status hth_batch_graph_check(hth_batch_graph *graph, hipStream_t stream);

/* Release a graph and its workspace (after its launches have completed).
   Null is accepted. */
hth_status hth_batch_graph_free(hth_batch_graph *graph);

/* hth_hash_batch without allocation, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, values and errors as
   hth_hash_batch; the call itself allocates nothing: the planning arrays and
   cross-task sums live in one static device array per GPU
   (HTH_NOALLOC_SCRATCH_BYTES, held from the first call on a device until the
   process ends; that first call also enqueues a kernel that clears it).
   Limits: count <= HTH_NOALLOC_MAX_COUNT (HTH_E_TOO_LARGE otherwise).  A
   batch whose plan does not fit the array (more than about 10^14 bytes of
   strings, reachable only with overlapping strings) produces no output, and
   hth_batch_check on the same stream reports HTH_E_TOO_LARGE.
   All calls on one GPU share its array: calls that overlap on one GPU (on
   different streams, or different host threads without ordering) race and
   give wrong values.  Order them on one stream. */
#define HTH_NOALLOC_MAX_COUNT 65536
#define HTH_NOALLOC_SCRATCH_BYTES 7406592
hth_status hth_hash_batch_noalloc(const hth_seed *seed, const uint8_t *bytes, const uint64_t *offsets,
                                  const uint64_t *lengths, uint64_t count, uint8_t *out, uint32_t out_width,
                                  hipStream_t stream);

/* Pre-size the workspace of `stream` for batches of up to max_count strings.
   Synchronous with respect to the host.  Errors: HTH_E_OOM, HTH_E_HIP. */
hth_status hth_reserve(uint64_t max_count, hipStream_t stream);

/* Synchronise `stream` and report whether the last batch on it was planned:
   HTH_OK, or HTH_E_TOO_LARGE if the device rejected its size (the batches of
   hth_hash_batch on this stream, and of hth_hash_batch_noalloc when its
   last call on the current device was on this stream). */
hth_status hth_batch_check(hipStream_t stream);

/* Diagnostic: a plain streaming read of `bytes` (rounded down to 16-byte
   pieces) of the device buffer buf (16-byte aligned), the achievable HBM
   read rate that the hashing kernel is measured against.  Each single-wave
   workgroup reads a contiguous share with non-temporal 16-byte loads, 4
   workgroups per compute unit (the rate is highest there), at most one
   workgroup per word of the device array sink (sink_words >= 1; its words
   are XOR-ed with the data read, so the caller zeroes it first).
   Enqueued on `stream`.  Errors: HTH_E_INVALID, HTH_E_HIP. */
hth_status hth_read_probe(const void *buf, uint64_t bytes, uint64_t *sink, uint32_t sink_words,
                          hipStream_t stream);

/* Tuning of the batched kernel for one output width; applies to later calls.
   waves_per_cu: resident single-wave workgroups per compute unit of the
   persistent grid (0 = the default, 8, or the occupancy limit if lower).  A task covers
   128 * 8^j full EHC executions of one string; the planner picks j in
   [min_task_level, max_task_level] (defaults 0 and 5): the coarsest level that
   still gives two tasks per resident wave, finer only if the workspace
   requires.  Setting both levels equal forces one task size.
   Errors: HTH_E_INVALID (bad width, min > max, max > 5). */
hth_status hth_set_tuning(uint32_t out_width, uint32_t waves_per_cu, uint32_t min_task_level,
                          uint32_t max_task_level);

/* ------------------------------------------------------------------------ */
/* Streaming: one string hashed from pieces appended over time.  The value  */
/* equals hth_hash_batch's for the concatenation of all pieces.  The state  */
/* is the tree stack of Eq. (3) (at most 7 pending items of k x b words per */
/* level) plus the bytes of the execution being filled, kept on the device; */
/* it can be saved to host memory and loaded into another stream (resume).  */
/* A stream object is used by one thread at a time.                          */
/* ------------------------------------------------------------------------ */

typedef struct hth_stream hth_stream;

/* Create an empty stream for `seed` (its family) and out_width.  Allocates
   its device state (about 0.8 MB), a planning workspace and a HIP stream of
   its own (default priority, for hth_stream_update_gather); synchronous.
   The seed must outlive the stream.  Errors: HTH_E_INVALID (null pointer,
   bad out_width, seed on another device), HTH_E_OOM, HTH_E_HIP. */
hth_status hth_stream_create(const hth_seed *seed, uint32_t out_width, hth_stream **out);

/* Append `len` bytes at device pointer `bytes` (any alignment), enqueued on
   `stream`; the bytes must stay valid until that work completes.  Every
   call on one hth_stream must be ordered (the same HIP stream, or
   synchronised).  len == 0 is a no-op.  Works as hth_stream_update_gather
   with one piece (its last kernel on the stream object's own stream); an
   update that completes no execution is one copy onto the carried bytes.
   Errors: HTH_E_INVALID (nothing enqueued), HTH_E_HIP (the state may be
   partly advanced: reset or load it before further use). */
hth_status hth_stream_update(hth_stream *st, const uint8_t *bytes, uint64_t len, hipStream_t stream);

/* Append `count` pieces in order: the same state as `count` calls of
   hth_stream_update, with the blocks of up to 64 pieces hashed in one
   launch (fewer when their block tables pass 1024 entries; the executions
   that straddle two pieces are assembled in the stream's state and hashed in
   the same launch).  A piece of a few hundred MB leaves most of the device
   idle on its own (the tree of Eq. (3) is cut into aligned blocks of 8^L
   executions, each hashed by whole passes of 128 executions, 256 for b = 4);
   gathered, the pieces fill it together.  pieces[i] is a device pointer to lens[i] bytes
   (any alignment; lens[i] == 0 is skipped), the pieces may lie in different
   allocations; both host arrays are read during the call, the bytes by the
   work enqueued on `stream` (valid until it completes).  Same ordering rule
   as hth_stream_update.  Each group's last kernel (the one that folds its
   results into the stream's state, reading no caller bytes) runs on a HIP
   stream of the stream object's own, beside the next group's work, ordered
   by events; every other call on the object waits for it where it must,
   and hth_stream_free synchronises it (under stream capture it runs on
   `stream`).  Errors: HTH_E_INVALID (null stream, null arrays with count >
   0, null piece of non-zero length; nothing enqueued), HTH_E_HIP (as for
   hth_stream_update). */
hth_status hth_stream_update_gather(hth_stream *st, const uint8_t *const *pieces, const uint64_t *lens,
                                    uint32_t count, hipStream_t stream);

/* Write the out_width-byte hash of everything appended so far to device
   pointer `out` (enqueued on `stream`).  The stream is unchanged and can
   take more updates.  Errors: HTH_E_INVALID, HTH_E_HIP. */
hth_status hth_stream_final(hth_stream *st, uint8_t *out, hipStream_t stream);

/* Back to the empty string (enqueued on `stream`). */
hth_status hth_stream_reset(hth_stream *st, hipStream_t stream);

/* Checkpoint: copy the state to host memory (synchronous on `stream`).
   With host == NULL, *size receives the bytes needed; otherwise *size is
   the buffer's size on entry (HTH_E_TOO_LARGE if too small) and the bytes
   written on return. */
hth_status hth_stream_save(hth_stream *st, void *host, size_t *size, hipStream_t stream);

/* Resume: load a state saved from a stream of the same width and family
   (synchronous on `stream`).  Errors: HTH_E_INVALID (not a saved state,
   other width or family, truncated, or a state that appending cannot
   produce: a stack level whose item count is not the matching base-8 digit
   of the execution count, or a byte count other than executions times the
   execution size plus the carried bytes; checked before any copy),
   HTH_E_HIP. */
hth_status hth_stream_load(hth_stream *st, const void *host, size_t size, hipStream_t stream);

/* Bytes appended so far (0 for null). */
uint64_t hth_stream_length(const hth_stream *st);

/* Free a stream (after its enqueued work completed; waits for its own
   internal stream).  Null is accepted. */
hth_status hth_stream_free(hth_stream *st);

/* ------------------------------------------------------------------------ */
/* Serving loop.  Hash requests arrive one at a time as host bytes; a       */
/* server admits them by device memory, gathers whatever has arrived into   */
/* batches (continuous batching: a batch leaves as soon as a stream slot is */
/* free) and hashes every batch with the planner and kernel of             */
/* hth_hash_batch, so a request's value does not depend on what it was     */
/* batched with.  A thread per stream slot does the scheduling.             */
/* ------------------------------------------------------------------------ */

typedef struct hth_server hth_server;

typedef struct hth_serve_config {
  uint64_t max_device_bytes;   /* device memory for request bytes in flight: the
                                  admission budget (0: 1 GiB) */
  uint64_t host_stage_bytes;   /* pinned host staging for submitted bytes (0: 1 GiB) */
  uint64_t max_request_bytes;  /* larger requests are refused (0: 16 MiB); must fit
                                  both of the above */
  uint64_t max_batch_bytes;    /* a batch stops growing at this many bytes
                                  (0: 64 MiB, at most 2^36) */
  uint32_t max_batch_requests; /* and at this many requests (0: 16384, at most 2^22) */
  uint32_t slots;              /* batches in flight, one stream each (0: 3, at most 8) */
  uint32_t max_outstanding;    /* submitted requests whose results are not yet
                                  collected (0: 2^20, at most 2^24; rounded up
                                  to a power of two) */
  uint32_t reserved;           /* set to 0 */
} hth_serve_config;

typedef struct hth_serve_report {
  uint64_t submitted;   /* requests accepted by submit */
  uint64_t completed;   /* results visible to poll/wait */
  uint64_t deferred;    /* requests that had to wait for device memory */
  uint64_t busy;        /* submits refused with HTH_E_BUSY */
  uint64_t batches;     /* batches hashed */
  uint64_t bytes;       /* request bytes hashed */
  double elapsed_s;     /* first submit to last completion */
  double gbps;          /* bytes / elapsed_s, in 10^9 bytes per second */
  double latency_p50_us, latency_p99_us, latency_max_us, latency_mean_us;
                        /* submit -> result visible, over completed requests */
  double mean_batch_requests;
} hth_serve_report;

/* Create a server on the current device for `seed` (which must outlive it).
   Allocates the device budget, the pinned staging (every page touched once,
   so that submits do not fault on them), per-slot streams and workspaces,
   and starts one thread per slot.  Unset (zero) fields take the
   defaults above.  Errors: HTH_E_INVALID (null pointer, limits out of range
   or inconsistent, seed on another device), HTH_E_OOM, HTH_E_HIP. */
hth_status hth_serve_create(const hth_serve_config *config, const hth_seed *seed, hth_server **out);

/* Submit one request: `len` bytes at host pointer host_bytes (copied before
   the call returns; the caller may reuse the memory), hashed to out_width
   (16, 24, 32 or 40) bytes.  *ticket receives the request's ticket.
   The request waits in the queue while the device budget is full (counted
   as deferred).  Errors: HTH_E_TOO_LARGE (len > max_request_bytes),
   HTH_E_BUSY (staging full or max_outstanding results uncollected: retry
   later), HTH_E_INVALID, HTH_E_HIP (the server stopped after an error). */
hth_status hth_serve_submit(hth_server *server, const void *host_bytes, uint64_t len, uint32_t out_width,
                            uint64_t *ticket);

/* Submit one request whose bytes stay in the caller's pinned host memory
   (hipHostMalloc, or a pinned torch tensor): nothing is copied at submit;
   the server's batch copies them to the device directly.  The caller must
   leave the `len` bytes unchanged and allocated until the ticket's result
   has been collected.  Requests submitted back to back from consecutive
   bytes are copied to the device together.  Otherwise as hth_serve_submit
   (HTH_E_BUSY only for max_outstanding: no staging is used).  For callers
   whose requests already arrive in pinned memory (e.g. network receive
   buffers), the submit path without the staging copy. */
hth_status hth_serve_submit_pinned(hth_server *server, const void *pinned_bytes, uint64_t len, uint32_t out_width,
                                   uint64_t *ticket);

/* Collect a result without blocking: HTH_OK copies out_width bytes to
   out_host and retires the ticket; HTH_E_BUSY means not ready yet;
   HTH_E_INVALID for an unknown or already collected ticket. */
hth_status hth_serve_poll(hth_server *server, uint64_t ticket, uint8_t *out_host);

/* As hth_serve_poll, but blocks until the result is ready. */
hth_status hth_serve_wait(hth_server *server, uint64_t ticket, uint8_t *out_host);

/* hth_serve_wait for n tickets; result i goes to out_host + i * out_stride
   (out_stride >= 40). */
hth_status hth_serve_wait_many(hth_server *server, const uint64_t *tickets, uint64_t n, uint8_t *out_host,
                               uint32_t out_stride);

/* Load replay: submits request i (bytes base + offsets[i], lengths[i],
   width widths[i]) at arrival_ns[i] nanoseconds after the call starts,
   retrying while the server answers HTH_E_BUSY; tickets go to tickets[i].
   `threads` client threads (1..64) share the requests in chunks of 64
   consecutive ones (chunk c goes to thread c mod threads; each thread
   submits in request order), so copies into the staging overlap.  Returns after the last submit, not after completion;
   on an error other than BUSY the remaining requests are not submitted. */
hth_status hth_serve_replay(hth_server *server, const uint8_t *base, const uint64_t *offsets,
                            const uint64_t *lengths, const uint32_t *widths, const uint64_t *arrival_ns,
                            uint64_t n, uint32_t threads, uint64_t *tickets);

/* As hth_serve_replay, submitting with hth_serve_submit_pinned: base must
   be pinned host memory, unchanged until every result is collected. */
hth_status hth_serve_replay_pinned(hth_server *server, const uint8_t *base, const uint64_t *offsets,
                                   const uint64_t *lengths, const uint32_t *widths, const uint64_t *arrival_ns,
                                   uint64_t n, uint32_t threads, uint64_t *tickets);

/* Hold (paused != 0) or release (0) batching: while held, submitted
   requests queue up (within the staging and outstanding limits) and no new
   batch starts; batches already in flight complete.  For bursts that should
   leave together, and for draining a server without new device work. */
hth_status hth_serve_pause(hth_server *server, int32_t paused);

/* Counters and latency percentiles since creation or the last reset. */
hth_status hth_serve_stats(hth_server *server, hth_serve_report *out);
hth_status hth_serve_reset_stats(hth_server *server);

/* Stop the slot threads (after the batches in flight complete) and free the
   server; uncollected results are dropped.  Null is accepted. */
hth_status hth_serve_destroy(hth_server *server);

#ifdef __cplusplus
}
#endif
#endif
