/*
 * hj.h -- C ABI of an MI355X (gfx950) equi hash join library.
 *
 * The operation (Section 3.1, "Fine-grained Steps in Hash Joins"): given two
 * relations R and S of <key, rid> tuples (two 4-byte integers each, Section
 * 5.1), R the build side and S the probe side, produce every pair
 * (rid_R, rid_S) whose tuples carry equal keys (Algorithm 1, step p4), and the
 * number of such pairs.  Two forms are offered, as in the paper:
 *   HJ_SHJ  simple hash join: build one table over all of R, probe it with S
 *           (Algorithm 1);
 *   HJ_PHJ  radix-partitioned hash join: split R and S into 2^B partitions on
 *           B low bits of the key's hash, in one or two passes, then join each
 *           partition pair (Algorithm 2, Section 3.1).
 * The number of passes and the radix bits of each pass are parameters, as the
 * paper tunes them to the memory hierarchy (Section 3.1).
 *
 * Conventions shared by every call:
 *  - All relation and output buffers are DEVICE pointers owned by the caller;
 *    the library never allocates device memory.  Scratch space comes from the
 *    caller's workspace (size from hj_workspace_bytes).
 *  - Relations are structure-of-arrays: key[n] and rid[n], int32, n < 2^31.
 *    Any int32 value is a legal key (no sentinel key); duplicates are allowed
 *    on both sides and produce cnt_R(k) * cnt_S(k) pairs for key k.
 *  - R is always the build side, even when |R| > |S|; the output columns are
 *    therefore fixed: rid_r[i] comes from R, rid_s[i] from S.
 *  - Output order is unspecified; the result is a multiset of pairs.
 *  - Calls are asynchronous on the given HIP stream (a hipStream_t passed as
 *    void*, NULL = the null stream) unless named *_sync.  Inputs must stay
 *    alive and unmodified until the stream has passed the call.  hj_join does
 *    no host synchronisation and no host<->device copy, so it can be captured
 *    into a HIP graph.
 *  - Every call returns an hj_status.  Argument validation happens on the host
 *    before any launch; on an error nothing is launched and hj_last_error()
 *    (thread-local) describes the cause.
 *  - The library holds no global mutable state apart from that thread-local
 *    message and a per-device attribute cache; concurrent calls on different
 *    streams with different workspaces are safe.
 */
#ifndef HJ_H
#define HJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hj_status {
    HJ_OK = 0,
    HJ_ERR_INVALID = 1,     /* bad argument (NULL buffer with n > 0, bad bits/passes, n >= 2^31) */
    HJ_ERR_CAPACITY = 2,    /* *_sync only: more pairs than out->capacity; the count is still reported */
    HJ_ERR_WORKSPACE = 3,   /* ws_bytes below hj_workspace_bytes(), or ws NULL */
    HJ_ERR_DEVICE = 4,      /* a HIP runtime call failed, or the device reported a failure in the
                               workspace's error word (hj_workspace_status); see hj_last_error() */
    HJ_ERR_UNSUPPORTED = 5  /* a parameter combination the library does not implement */
} hj_status;

/* HJ_AUTO: the library evaluates its cost model (hj_model_seconds) for SHJ, for
   PHJ without partitioning (|R| <= 8192), and for PHJ in one or two radix
   passes around 4096 R tuples per partition with both partitioning tiles (one
   tile when p->tile is set), and runs the plan with the least modelled time;
   hash, lds_cap and flags are kept.  hj_resolve_params shows the choice. */
typedef enum hj_algo { HJ_SHJ = 0, HJ_PHJ = 1, HJ_AUTO = 2 } hj_algo;

/* Hash applied to a key before its radix bits are taken (Section 3.1 partitions
   on the low bits of the integer hash value).  The join result does not depend
   on it; it only changes which partition a tuple lands in. */
typedef enum hj_hash {
    HJ_HASH_IDENTITY = 0,   /* the key's own bits */
    HJ_HASH_MURMUR2 = 1     /* MurmurHash 2.0 of the key's 4 bytes (the paper's choice, Section 5.1) */
} hj_hash;

/* A relation: `n` tuples, device arrays key[n] and rid[n] (int32). */
typedef struct hj_rel {
    const int32_t* key;
    const int32_t* rid;
    uint64_t n;
} hj_rel;

/* The result buffers: device arrays rid_r[capacity] and rid_s[capacity].
   Pair i is (rid_r[i], rid_s[i]).  When the join has more pairs than
   `capacity`, no element at or beyond `capacity` is written and the contents
   of [0, capacity) are unspecified. */
typedef struct hj_out {
    int32_t* rid_r;
    int32_t* rid_s;
    uint64_t capacity;
} hj_out;

/* Output in one pass: each workgroup counts its pairs, reserves that many
   output slots with one atomic add on the running total, then writes them
   (Section 3.3's block allocator, one block per workgroup), instead of a count
   pass, a scan and a write pass.  Same multiset of pairs.  Applies to SHJ and
   PHJ. */
#define HJ_FLAG_ONE_PASS 1u

/* Join parameters.
   algo    HJ_SHJ, HJ_PHJ or HJ_AUTO.
   passes  PHJ: number of radix passes, 1 or 2; or 0 = no partitioning, for
           |R| <= 8192: R is one LDS-resident table probed by every S chunk
           (ignored by SHJ).
   bits    PHJ: radix bits of pass 1 and pass 2.  B = bits[0] (+ bits[1] when
           passes == 2) must be in 1..20 and each used entry in 1..13.  The
           2^B partitions are the values of the B low bits of the hash; pass 1
           splits on the high bits[0] of them, pass 2 on the low bits[1].
   hash    an hj_hash value.
   tile    tuples per partitioning tile: a power of two in 1024..8192, or 0
           = chosen from the sizes (8192 when |R| + |S| >= 2^25, or >= 2^24
           with one pass of 8 or more bits; else 4096).
   lds_cap largest R partition (tuples) joined from an LDS-resident table:
           0 = chosen from |R| and B; else a multiple of 64 in 256..8192.
           Larger partitions take the HBM-table path.
   flags   0 or HJ_FLAG_ONE_PASS. */
typedef struct hj_params {
    uint32_t algo;
    uint32_t passes;
    uint32_t bits[2];
    uint32_t hash;
    uint32_t tile;
    uint32_t lds_cap;
    uint32_t flags;
} hj_params;

/* Fills `p` with the library defaults: PHJ, 2 passes of 6 bits, identity hash,
   tile and lds_cap chosen from the sizes, two-pass output. */
void hj_default_params(hj_params* p);

/* Copies `p` into `out` with every value the library chooses from the sizes
   filled in, as hj_join would use it for |R| = n_r, |S| = n_s: PHJ tile and
   lds_cap (and HJ_FLAG_ONE_PASS for passes == 0, which always writes its output
   in one pass).  Host only.  Returns HJ_ERR_INVALID for invalid parameters. */
hj_status hj_resolve_params(const hj_params* p, uint64_t n_r, uint64_t n_s, hj_params* out);

/* The cost model of Section 4 (Eq. 2-3) as calibrated on MI355X: the predicted
   elapsed time of hj_join with parameters p (HJ_AUTO resolved first) for
   |R| = n_r, |S| = n_s and `pairs` output pairs, in seconds.  Every kernel
   launch of the plan is one step, timed as the delay of a dependent launch,
   the kernel's ramp-up and drain, and the larger of its memory time
   (algorithmic bytes over the bandwidth of its access pattern) and its
   workgroup latency (rounds of resident workgroups times one workgroup's
   duration).  Host only; the constants come from per-kernel timings of a grid
   of joins on the device. */
hj_status hj_model_seconds(const hj_params* p, uint64_t n_r, uint64_t n_s, uint64_t pairs, double* seconds);

/* Bytes of device workspace hj_join needs for these parameters and sizes.
   Returns 0 if the parameters are invalid (hj_last_error() says why). */
size_t hj_workspace_bytes(const hj_params* p, uint64_t n_r, uint64_t n_s);

/* Joins R and S into `out` (Algorithm 1 for SHJ, Algorithm 2 for PHJ).
   ws/ws_bytes: device workspace of at least hj_workspace_bytes(p, R->n, S->n)
   bytes, 256-byte aligned, not used by any other call in flight.
   d_count: device pointer to one uint64; always receives the total number of
   pairs, also when it exceeds out->capacity.
   Asynchronous on `stream`; returns after enqueueing the work. */
hj_status hj_join(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out,
                  void* ws, size_t ws_bytes, uint64_t* d_count, void* stream);

/* hj_join followed by a synchronisation of `stream` and a copy of the count
   into *h_count.  Returns HJ_ERR_DEVICE when the join's device error word is
   set (see hj_workspace_status), else HJ_ERR_CAPACITY when
   *h_count > out->capacity. */
hj_status hj_join_sync(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out,
                       void* ws, size_t ws_bytes, uint64_t* d_count, uint64_t* h_count,
                       void* stream);

/* Per-kernel timing of one hj_join: each launch is bracketed with HIP events
   recorded on `stream`; the call synchronises the stream before returning.
   names[i] (static strings) and ms[i] describe launch i, for at most
   max_launches launches; *n_launches receives the number of launches made. */
hj_status hj_join_timed(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out,
                        void* ws, size_t ws_bytes, uint64_t* d_count, void* stream,
                        const char** names, float* ms, uint32_t max_launches,
                        uint32_t* n_launches);

/* hj_join without a workspace argument, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc).  The workspace is a fixed array of this library in device
   memory: 64 MiB (67,108,864 bytes) on every GPU the library runs on, held from
   the first call on that GPU until the process ends.  Arguments, result and
   asynchrony as hj_join; nothing is allocated.  Returns HJ_ERR_WORKSPACE,
   before touching the device, when hj_workspace_bytes(p, R->n, S->n) exceeds
   the array (e.g. HJ_AUTO up to about |R| = |S| = 1.7M tuples, SHJ up to about
   3M + 3M).  All calls on one GPU share its array: calls that overlap on one
   GPU (two streams, two threads) race; serialise them.  The call's device
   error word (hj_workspace_status) sits in the array and is not reachable by
   the caller. */
hj_status hj_join_noalloc(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out,
                          uint64_t* d_count, void* stream);

/* ---- Build once, probe many times -----------------------------------------
   The two phases of Algorithm 1 as separate calls: hj_build makes R's
   build-side structure once, and any number of hj_probe calls join relations
   S against it (concurrently too, each with its own workspace).  For SHJ the
   table is the hash table over R (steps b1-b4); for PHJ with 1 or 2 passes it
   is R partitioned with the radix passes of Algorithm 2 plus the range of
   every partition, so a probe partitions only S and joins the partition
   pairs (each R partition's LDS table is rebuilt inside the join kernel, as
   in hj_join); for PHJ with passes 0 nothing is stored and probes read R.
   The result of a probe is the result hj_join would give for (R, S) with the
   table's parameters. */

/* A table over R, filled in by hj_build.  The caller keeps the structure, its
   build workspace and (for SHJ and for PHJ with passes 0) R's arrays alive
   and unmodified while probes may use it. */
typedef struct hj_table {
    hj_params params;      /* as run: HJ_AUTO and the size-dependent choices resolved */
    uint64_t n_r;          /* tuples of R */
    const int32_t* r_key;  /* R's columns as given to hj_build.  SHJ probes and PHJ */
    const int32_t* r_rid;  /*   probes with passes 0 read both: the rids of matches,
                              and the keys when S tuples meet a duplicate-heavy key
                              (its matches are found by scanning R's key column);
                              hj_probe rejects a NULL column there.  PHJ probes with
                              1 or 2 passes read neither. */
    void* ws;              /* the build workspace that holds the table */
    size_t ws_bytes;
} hj_table;

/* Bytes of device workspace hj_build needs for a table over n_r tuples (the
   table lives there).  0 if the parameters are invalid. */
size_t hj_table_bytes(const hj_params* p, uint64_t n_r);

/* Builds the table over R into ws (256-byte aligned, >= hj_table_bytes) and
   fills *table.  Size-dependent parameters (tile 0, lds_cap 0, HJ_AUTO) are
   chosen from |R| alone.  Asynchronous on `stream`; probes must be ordered
   after it (same stream, or an event). */
hj_status hj_build(const hj_params* p, const hj_rel* R, void* ws, size_t ws_bytes, void* stream,
                   hj_table* table);

/* Bytes of device workspace hj_probe needs for a probe of n_s tuples. */
size_t hj_probe_workspace_bytes(const hj_table* table, uint64_t n_s);

/* Joins S against the table: output, count and capacity behaviour as in
   hj_join.  ws: >= hj_probe_workspace_bytes(table, S->n) bytes, 256-byte
   aligned, not used by any other call in flight (the table itself is only
   read).  Asynchronous on `stream`. */
hj_status hj_probe(const hj_table* table, const hj_rel* S, const hj_out* out, void* ws, size_t ws_bytes,
                   uint64_t* d_count, void* stream);

/* ---- Batched joins ------------------------------------------------------
   Many independent joins of uneven sizes enqueued together.  A plan fixes the
   jobs (pointers and sizes) and the per-job parameters; running it enqueues
   every job on the given stream.  Jobs with PHJ and passes == 0 (R fits one
   LDS table) run together in one multi-job kernel; the others run their own
   launch sequences on 16 concurrent lanes whose workspace slices are reused
   job after job.  Unless HJ_BATCH_NO_GRAPH is set, the first run with a given
   workspace captures the whole batch into one HIP graph (on a stream of the
   plan) and every run launches that graph on the caller's stream. */

/* One join of a batch: R, S, its output buffers and a device uint64 count. */
typedef struct hj_job {
    hj_rel R;
    hj_rel S;
    hj_out out;
    uint64_t* d_count;
} hj_job;

typedef struct hj_batch_plan hj_batch_plan;

/* Enqueue the batch directly on the streams instead of through a HIP graph. */
#define HJ_BATCH_NO_GRAPH 1u

/* Creates a plan for `njobs` jobs (host array, copied).  params: host array of
   njobs parameter sets, or NULL for the library's choice per job (HJ_AUTO with
   HJ_FLAG_ONE_PASS: the plan the cost model rates fastest).  Pointers inside the jobs must stay valid while the plan
   is used.  Allocates pinned host memory and creates streams and events; no
   device memory. */
hj_status hj_batch_plan_create(uint32_t njobs, const hj_job* jobs, const hj_params* params, uint32_t flags,
                               hj_batch_plan** plan);

/* Device workspace bytes hj_batch_run needs for this plan. */
size_t hj_batch_workspace_bytes(const hj_batch_plan* plan);

/* Number of jobs of the plan that run in the multi-job direct kernel. */
uint32_t hj_batch_direct_jobs(const hj_batch_plan* plan);

/* Nodes (kernels, copies, event records and waits) of the HIP graph the plan
   captured at its first graph run; 0 before that or with HJ_BATCH_NO_GRAPH. */
size_t hj_batch_graph_nodes(const hj_batch_plan* plan);

/* Enqueues every job of the plan on `stream` (asynchronous).  Each job's
   d_count receives its pair count; a job whose count exceeds its capacity
   writes nothing past its capacity. */
hj_status hj_batch_run(hj_batch_plan* plan, void* ws, size_t ws_bytes, void* stream);

void hj_batch_plan_destroy(hj_batch_plan* plan);

/* One-shot batch: the plan of hj_batch_plan_create run once without a graph
   (params as there), then freed.  Synchronises `stream` before returning.
   ws: >= hj_batch_bytes(njobs, jobs, params) bytes, 256-byte aligned. */
size_t hj_batch_bytes(uint32_t njobs, const hj_job* jobs, const hj_params* params);
hj_status hj_batch(uint32_t njobs, const hj_job* jobs, const hj_params* params, void* ws, size_t ws_bytes,
                   void* stream);

/* ---- Serving ------------------------------------------------------------
   A server accepts join requests as they arrive (from any thread) and runs
   them with continuous batching: a dispatcher thread owns `slots` streams;
   whenever a slot is idle it admits waiting requests, first come first
   served, while the summed footprints of all requests on the device stay
   within mem_cap_bytes, and runs them there as one batch (requests with PHJ
   and passes == 0 together in the multi-job direct kernel, the others one
   after another).  Batches on different slots overlap on the device, and a
   finished batch frees its footprint and its slot for the next requests.
   The server's device workspace (split evenly between the slots) comes from
   the caller; the inputs of every request stay resident in device memory
   until the request completes. */

typedef struct hj_server hj_server;

typedef struct hj_server_config {
    uint64_t mem_cap_bytes;   /* admission cap on the summed request footprints */
    uint32_t slots;           /* concurrent batches (streams), 1..16 */
    uint32_t max_batch_jobs;  /* requests admitted into one batch */
    uint32_t flags;           /* must be 0 */
} hj_server_config;

/* Starts a server.  ws: device workspace (256-byte aligned) shared by the
   slots; a request whose hj_workspace_bytes exceeds a slot's share is
   rejected.  Creates streams, events, pinned host staging and one thread. */
hj_status hj_server_create(const hj_server_config* cfg, void* ws, size_t ws_bytes, hj_server** server);

/* Queues one request (thread-safe, returns at once).  footprint: the bytes the
   request holds on the device while admitted (inputs, output, workspace), as
   the caller accounts them; admission uses the larger of that and the bytes
   the server accounts itself: 8 per tuple of R and S, 8 per output slot of
   out.capacity, the count and the request's workspace (hj_workspace_bytes).
   *ticket identifies it in hj_server_poll. */
hj_status hj_server_submit(hj_server* server, const hj_job* job, const hj_params* params, uint64_t footprint,
                           uint64_t* ticket);

/* Queues a probe of a resident table (hj_build) by S (thread-safe, returns at
   once): the request runs hj_probe on a slot, so relations and their tables
   built once stay on the device and serve many requests.  The table and
   everything it points to must stay alive until the request has finished.
   footprint: as for hj_server_submit, with the server's own account over S,
   the output and the probe workspace (the table is the caller's). */
hj_status hj_server_submit_probe(hj_server* server, const hj_table* table, const hj_rel* S, const hj_out* out,
                                 uint64_t* d_count, uint64_t footprint, uint64_t* ticket);

/* Moves up to `max` finished requests out of the server: ticket, status
   (HJ_OK, HJ_ERR_CAPACITY if rejected by admission, HJ_ERR_DEVICE), seconds
   from submission to completion and from submission to admission.  *n gets
   the number returned.  Returns a device error if the server has stopped. */
hj_status hj_server_poll(hj_server* server, uint64_t* tickets, int32_t* status, double* latency_s,
                         double* queue_s, uint32_t max, uint32_t* n);

/* Blocks until every submitted request has finished. */
hj_status hj_server_drain(hj_server* server);

/* Counters: requests completed and rejected, batches launched, footprint bytes now admitted. */
hj_status hj_server_stats(hj_server* server, uint64_t* completed, uint64_t* rejected, uint64_t* batches,
                          uint64_t* bytes_in_use);

/* Finishes the queued requests, stops the dispatcher and frees the server. */
void hj_server_destroy(hj_server* server);

/* ---- Relations in host memory, larger than the device ---------------------
   The paper's joins of datasets beyond its zero-copy buffer (appendix "More
   Experimental Results", "Large datasets that cannot fit into the zero copy
   buffer"), as an external-memory hash join with device memory as the main
   memory: R, then S, streams through the device in chunks that are split into
   2^k partitions on k high bits of the key's MurmurHash 2.0 (the radix passes
   of Algorithm 2) and copied back to host memory; the partitions of all chunks
   are linked into partition pairs, and each pair is copied to the device and
   joined with `p` (any hj_params, HJ_AUTO recommended); its pairs are copied to
   the host output.  k is the smallest fan-out whose expected largest pair fits
   the workspace (k = 0: no partition pass, the whole join runs on the device).
   An S partition too large for the device with its R partition, or whose pairs
   overflow the device output room, is joined in pieces against the whole R
   partition.  Result as hj_join (multiset of pairs, count in *h_count,
   HJ_ERR_CAPACITY when it exceeds out->capacity, nothing written past it).
   R, S and out are HOST pointers (pinned memory from hipHostMalloc copies
   asynchronously; pageable memory works, more slowly).  ws: device workspace
   of at least 64 MiB, 256-byte aligned; its size bounds the device memory the
   call uses.  Synchronous: returns when the output is in host memory.
   Allocates a pinned host buffer of 8 (|R| + |S|) bytes for the partitions and
   two streams for the call's duration; no device memory.  Returns
   HJ_ERR_WORKSPACE when one R partition with its join does not fit the
   workspace (a key with that many duplicates). */
typedef struct hj_external_info {
    uint32_t fanout_bits;   /* partitions of the out-of-core pass: 2^fanout_bits (0: none) */
    uint32_t pieces;        /* device joins run (partition pairs, or pieces of them) */
    uint64_t chunk_tuples;  /* tuples per chunk of the partition pass */
    double partition_s;     /* wall time of the partition pass, copies included */
    double join_s;          /* wall time of joining the partition pairs, copies included */
    double total_s;         /* wall time of the call */
    uint64_t h2d_bytes;     /* bytes copied host -> device */
    uint64_t d2h_bytes;     /* bytes copied device -> host */
} hj_external_info;

hj_status hj_join_external(const hj_params* p, const hj_rel* R, const hj_rel* S, const hj_out* out, void* ws,
                           size_t ws_bytes, uint64_t* h_count, hj_external_info* info);

/* Device-side failures of an asynchronous call.  Every workspace handed to
   hj_join, hj_build, hj_probe, hj_batch_run or a server starts with an 8-byte
   error word that the call's first kernel clears.  The chained (decoupled
   look-back) scans that place partitions and output wait on their
   predecessors with a bounded number of polls; a wait that runs out ends its
   kernel normally and sets a bit there, and the call's output is then not
   valid.  This call synchronises `stream` and returns HJ_OK when the error
   word of `ws` (the workspace of the last call on that stream) is clear, else
   HJ_ERR_DEVICE with the cause in hj_last_error().  hj_join_sync checks it by
   itself; a server marks the requests of such a batch HJ_ERR_DEVICE.
   Failure injection for tests of these paths: the environment variable
   HJ_DEBUG_FAIL_PHASE, read at every call, set to "scan_stall" makes the first
   tile of every histogram and count scan withhold its status (the waits give
   up after 64 polls), and set to "launch:<phase>" (e.g. "launch:part_scatter") makes that
   launch report a launch failure (HJ_ERR_DEVICE from the call). */
hj_status hj_workspace_status(const void* ws, void* stream);

/* Static description of a status code. */
const char* hj_status_str(hj_status s);

/* Thread-local description of the last error returned on this thread ("" if none). */
const char* hj_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
uint32_t hj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HJ_H */
