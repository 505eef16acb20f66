/*
 * pivco.h -- C ABI of the MI355X (gfx950) PivCo-Huffman codec.
 *
 * PivCo-Huffman (Zukowski, 2026) stores a Huffman-coded block "pivoted": every
 * internal node of the (length-limited, canonical) code tree keeps one bitmap
 * with one bit per symbol that passes through it, in stream order (Sec. 2,
 * Fig. 2-3).  Decoding merges the children's dense symbol sequences bottom-up
 * under control of each node's bitmap (Sec. 3); encoding splits the codes
 * top-down and emits the bitmaps (Sec. 4, Table 11).  Skewed nodes may be
 * entropy-coded instead of stored raw (Sec. 5); here with 32-lane interleaved
 * binary rANS with 12-bit probabilities (method of ref. [4] of the paper), or
 * with the selective tANS of Sec. 5.2 (50 static byte tables for bitmap
 * skews of 50..99%, 32 cursors per chunk, App. D's marker).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers (HIP device memory, e.g. the
 *     data_ptr() of a torch tensor); h_* are host pointers.  The caller owns
 *     every buffer; the library never frees caller memory.
 *   - Device inputs (d_in) must be 16-byte aligned.
 *   - Work is enqueued on the given stream and is asynchronous unless the
 *     comment says "synchronous".  Argument errors are returned at once;
 *     errors found in the data (corrupt stream, too small output) are written
 *     per job to d_status as a pivco_status value.
 *   - Decoding never reads outside [d_in, d_in + in_len) and never writes
 *     outside [d_out, d_out + out_cap), also on corrupt input.
 *   - Functions are thread-safe; a plan object may be used by one thread at a
 *     time.
 *
 * Stream format (v1, little-endian; layout written out in the library's
 * format notes): a 48-byte stream header, a table of block offsets, a table
 * of rANS scratch offsets, then blocks.  Each block holds its 4-bit code
 * lengths (128 bytes, App. D), one kind bit and one count of 1 bits per
 * internal node (breadth-first order), the raw bitmaps, then the rANS bodies.
 * A v2 stream (version 2) is the same with the flat-subtree tree of Sec.
 * 2.2.3-2.2.4 in every coded block: the symbols of each code length are cut
 * into power-of-two groups (largest first) and a group of 2^D >= 4 symbols is
 * one flat node, whose body holds a D-bit index into its group per passing
 * symbol (ceil(n_v D / 8) bytes, App. D).  Stream flags bit 0 (header bytes
 * 6-7) says that the entropy-coded nodes use the byte tANS tables instead of
 * rANS: such a body is marker u8 (table t = 1..50 for a majority-bit
 * fraction of (t + 49)%, | 0x80 when the bitmap is coded complemented) | 0 u8
 * | 0 u16 | body length u32, then per chunk of 2^chunk_log2 bits (>= 2^8)
 * 32 u16 cursor states, 32 u16 stream lengths, the 32 cursors' bit streams
 * (cursor l codes bytes l, l + 32, ... of the chunk) and zero padding to 4
 * bytes.  Every decode entry point reads v1 and v2 streams, with either
 * coder.
 */
#ifndef PIVCO_H
#define PIVCO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIVCO_OK = 0,
  PIVCO_E_ARG = -1,          /* bad argument (returned synchronously) */
  PIVCO_E_CAPACITY = -2,     /* output or workspace too small */
  PIVCO_E_CORRUPT = -3,      /* stream fails validation */
  PIVCO_E_UNSUPPORTED = -4,  /* valid stream outside this library's limits */
  PIVCO_E_DEVICE = -5,       /* HIP runtime error */
  PIVCO_E_BUDGET = -6        /* serving: request larger than the memory budget */
} pivco_status;

/* A code tree given by its 256 code lengths (0 = symbol absent).  Codes are
 * canonical: ordered by (length, symbol), first code 0 (ref. [5]). */
typedef struct {
  uint8_t code_len[256];
} pivco_tree;

typedef struct {
  uint32_t block_size;       /* symbols per block, >= 1 */
  uint32_t max_len;          /* code length limit; 11 as in App. D (8..12) */
  uint32_t ans_mode;         /* 0: raw bitmaps only; 1: rANS for nodes whose
                                one-bit fraction is < 0.1 or > 0.9;
                                2: rANS for every internal node (testing);
                                3: the selective byte tANS of Sec. 5.2 (a node
                                of >= 256 bits whose majority-bit fraction f
                                exceeds 0.625 takes table round(100 f) - 49 if
                                (depth + h) / (depth + 1) < 0.95, h the
                                table's expected bits per bit; stream flags
                                bit 0) */
  uint32_t rans_chunk_log2;  /* bits per entropy-coded chunk = 2^this; 16
                                (5..24; 8..24 with ans_mode 3) */
  const pivco_tree *tree;    /* NULL: one optimal tree per block from its
                                histogram; else this tree for every block */
  uint32_t tree_shape;       /* 0: canonical trees (a v1 stream); 1: the
                                flat-subtree trees of Sec. 2.2.3-2.2.4 built
                                from the same code lengths (a v2 stream) */
  uint32_t reserved;         /* 0 */
} pivco_encode_opts;

/* One decode job: a whole stream. */
typedef struct {
  const void *d_in;          /* stream, 16-byte aligned */
  uint64_t in_len;           /* bytes readable at d_in */
  void *d_out;               /* decoded bytes */
  uint64_t out_cap;          /* bytes writable at d_out */
} pivco_job;

/* ---------------------------------------------------------------------- */
/* Tree construction (host, synchronous)                                  */
/* ---------------------------------------------------------------------- */

/* Optimal code lengths limited to max_len bits for the given symbol counts
 * (App. D fixes the limit at 11 bits).  Package-merge, then the ascending
 * lengths are assigned to symbols ordered by (count desc, symbol asc).
 * E_ARG if fewer than two symbols have a nonzero count or max_len is out of
 * [1, 15] or too small for the alphabet. */
pivco_status pivco_build_tree(const uint64_t counts[256], uint32_t max_len, pivco_tree *out);

/* ---------------------------------------------------------------------- */
/* Encode (Sec. 4)                                                        */
/* ---------------------------------------------------------------------- */

/* Upper bound on the stream size for n input bytes. */
uint64_t pivco_encode_bound(uint64_t n, const pivco_encode_opts *o);

/* Device workspace bytes pivco_encode needs for n input bytes. */
uint64_t pivco_encode_workspace(uint64_t n, const pivco_encode_opts *o);

/* Encode n bytes at d_in into a v1 (or, with tree_shape 1, v2) stream at
 * d_out: histograms (Sec. 4: end-to-end encode is dominated by them),
 * length-limited optimal code lengths per block (package-merge on the
 * device, with the tie rules every encoder of the format follows: items by
 * weight, a single before a package on equal weight, symbols by id; the
 * multiset of lengths handed out ascending to the symbols by (count desc, id
 * asc)) or the supplied tree, the top-down split of Table 11, entropy coding
 * of the selected nodes, assembly.  The stream is byte-identical to the one
 * the format definition implies.  Synchronous: returns the stream length in
 * *h_out_len.  Errors: E_ARG (bad options or a supplied tree that misses a
 * symbol present in the data), E_CAPACITY (out_cap or ws_bytes too small;
 * nothing is written to d_out), E_UNSUPPORTED (ans_mode 3 with 2^24-bit
 * chunks only: a cursor's stream longer than its 16-bit length field),
 * E_DEVICE.  The tANS tables are copied to the device on their first use
 * (synchronously). */
pivco_status pivco_encode(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                          uint64_t *h_out_len, const pivco_encode_opts *o, void *d_ws,
                          uint64_t ws_bytes, hipStream_t s);

/* The same encode, asynchronous on s (nothing waits on the host, so it can
 * be captured in a HIP graph once the tANS tables are on the device): the
 * stream length goes to *d_out_len (a device uint64; the length the stream
 * needs also when it exceeds out_cap) and the call's status to *d_status (a
 * device int32: PIVCO_OK, E_ARG for a supplied tree that misses a present
 * symbol, E_CAPACITY when the stream exceeds out_cap -- then nothing is
 * written to d_out -- or E_UNSUPPORTED as above).  Argument errors are
 * returned at once.  Workspace and bound as for pivco_encode. */
pivco_status pivco_encode_async(const void *d_in, uint64_t n, void *d_out, uint64_t out_cap,
                                uint64_t *d_out_len, int32_t *d_status, const pivco_encode_opts *o,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s);

/* ---------------------------------------------------------------------- */
/* Decode (Sec. 3, bottom-up merge)                                       */
/* ---------------------------------------------------------------------- */

/* Header fields of a stream from a host copy of its first 48 bytes. */
pivco_status pivco_stream_info(const void *h_hdr, uint64_t hdr_len, uint64_t *n_total,
                               uint32_t *n_blocks, uint32_t *block_size, uint64_t *ans_words);

/* Device workspace bytes needed to decode these jobs.  Synchronous: reads
 * the stream headers from device memory.  Returns 0 on an argument error. */
uint64_t pivco_decode_workspace(const pivco_job *h_jobs, uint32_t count, hipStream_t s);

/* Decode every job in one batched launch: a persistent kernel takes blocks
 * from an atomic queue ordered by decreasing block size.  Synchronous up to
 * the point where kernels are enqueued (it reads the stream headers); the
 * decode itself runs asynchronously on s.  d_status[count] receives one
 * pivco_status per job. */
pivco_status pivco_decode_batch(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s);

/* One job; same as pivco_decode_batch with count = 1. */
pivco_status pivco_decode(const void *d_in, uint64_t in_len, void *d_out, uint64_t out_cap,
                          int32_t *d_status, void *d_ws, uint64_t ws_bytes, hipStream_t s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as pivco_decode, with its workspace in a fixed device array of
 * PIVCO_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  Allocates no device memory.  Returns E_CAPACITY,
 * before any device work, when the stream needs more workspace than that
 * (pivco_decode_workspace gives the need: about 5.6 KB per block plus rANS
 * scratch and the boundary tables of blocks of more than 64Ki symbols).  All
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (other streams or threads) race, so callers serialise them; the next call
 * may start once this one's work on s has completed or is ordered after it
 * on the same stream.  Otherwise as pivco_decode (synchronous up to the
 * kernel launches, which read the stream header).  A stream with tANS nodes
 * uses the library's static table arrays, copied to the GPU by the first
 * call that needs them (a copy, not an allocation). */
#define PIVCO_NOALLOC_SCRATCH_BYTES (32ull << 20)
pivco_status pivco_decode_noalloc(const void *d_in, uint64_t in_len, void *d_out, uint64_t out_cap,
                                  int32_t *d_status, hipStream_t s);

/* Baseline for comparison: the same kernel launched once per block, one
 * launch after the other on s (no persistent queue, no graph). */
pivco_status pivco_decode_plain(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                void *d_ws, uint64_t ws_bytes, hipStream_t s);

/* Ablation: the same decode with the top-down scheme of Sec. 2.1 instead of
 * the bottom-up merge of Sec. 3.  Per slice of 4096 outputs, every internal
 * node splits the positions that reach it by its bits, stably, into its
 * children's lists (partition), and a leaf writes its symbol at the
 * positions that reach it (scatter).  Same jobs, workspace, statuses and
 * validation as pivco_decode_batch; the decoded bytes are identical.  v2
 * streams (flat-subtree trees) get PIVCO_E_UNSUPPORTED. */
pivco_status pivco_decode_topdown(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                  void *d_ws, uint64_t ws_bytes, hipStream_t s);

/* Launch configuration of the batched decode, chosen by pivco_autotune. */
typedef struct {
  uint32_t merge_variant;    /* index into the compiled merge kernels */
  uint32_t merge_grid;       /* workgroups of the persistent merge kernel */
  uint32_t rans_grid;        /* workgroups of the rANS decode kernel */
  uint32_t grid_mode;        /* 0: persistent merge kernel over the work queue;
                                1: one non-persistent launch with a workgroup
                                per work item (merge_grid ignored) */
} pivco_tune;

/* Number of compiled merge-kernel variants and a short description of one. */
uint32_t pivco_merge_variants(void);
const char *pivco_merge_variant_name(uint32_t v);

/* A prepared batch: job table and work queue uploaded once, the decode
 * captured in a HIP graph; each launch replays the graph.  Creation is
 * synchronous.  tune may be NULL (default configuration). */
typedef struct pivco_batch_plan pivco_batch_plan;
pivco_status pivco_batch_plan_create(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                                     void *d_ws, uint64_t ws_bytes, const pivco_tune *tune,
                                     hipStream_t s, pivco_batch_plan **out);
pivco_status pivco_batch_plan_launch(pivco_batch_plan *p, hipStream_t s);
/* Record hEvents around the merge kernel only (no graph) for timing. */
pivco_status pivco_batch_plan_launch_timed(pivco_batch_plan *p, hipStream_t s,
                                           hipEvent_t merge_begin, hipEvent_t merge_end);
void pivco_batch_plan_destroy(pivco_batch_plan *p);

/* The fastest launch configuration for these jobs: every merge variant
 * (workgroup size, tile size of whole blocks, outputs per task) with three
 * persistent grid sizes, then the rANS grid (one, two or four workgroups per
 * CU) when the jobs have rANS nodes; each candidate is the best of three
 * timed batched decodes.  The choice is cached per device architecture and
 * workload bucket (work items per CU, mean symbols per item, share of tile
 * items, rANS present): a later call for the same bucket returns it without
 * timing.  Synchronous. */
pivco_status pivco_autotune(const pivco_job *h_jobs, uint32_t count, int32_t *d_status,
                            void *d_ws, uint64_t ws_bytes, hipStream_t s, pivco_tune *out);
/* Forgets every cached autotuner choice. */
void pivco_autotune_cache_clear(void);

/* ---------------------------------------------------------------------- */
/* PivCo-Golomb (App. G)                                                  */
/* ---------------------------------------------------------------------- */
/* The pivoted layout applied to a unary code (App. G): instead of a tree, a
 * list of bitmaps, one per code-bit position.  A value v (uint8) is coded as
 * v 0-bits and a 1-bit; bitmap k holds, in stream order, the k-th code bit of
 * every value >= k.  Stream format "PVG1" (little-endian): header 32 bytes
 * (magic, version 1, flags 0, n_total u64, block_size u32, n_blocks u32,
 * reserved u64), block offsets u64[n_blocks + 1], then per block (at a
 * multiple of 4 bytes) comp_size u32, n u32, K u16 (bitmaps: largest value
 * + 1), pad u16, the bitmap sizes n_1 .. n_{K-1} (u32), and the bitmaps
 * (ceil(n_k / 8) bytes each, LSB first, zero padding bits). */
uint64_t pivco_golomb_encode_bound(uint64_t n, uint32_t block_size);
uint64_t pivco_golomb_encode_workspace(uint64_t n, uint32_t block_size);
/* Encodes n values at d_in (synchronous; the stream length in *h_out_len).
 * E_ARG on bad arguments (d_out must be 16-byte aligned), E_CAPACITY when
 * out_cap or ws_bytes is too small. */
pivco_status pivco_golomb_encode(const void *d_in, uint64_t n, uint32_t block_size, void *d_out,
                                 uint64_t out_cap, uint64_t *h_out_len, void *d_ws, uint64_t ws_bytes,
                                 hipStream_t s);
/* Workspace for pivco_golomb_decode (reads the stream headers). */
uint64_t pivco_golomb_decode_workspace(const pivco_job *h_jobs, uint32_t count, hipStream_t s);
/* Decodes every job, one workgroup per block: bottom-up over the bitmap list
 * (at bitmap k a 1 bit gives 0, a 0 bit 1 + the next bitmap's value: the
 * merge_vec_cst_plus1 primitive), per job a status in d_status (E_CORRUPT
 * for a stream that fails validation, E_CAPACITY for a small output).
 * Synchronous. */
pivco_status pivco_golomb_decode(const pivco_job *h_jobs, uint32_t count, int32_t *d_status, void *d_ws,
                                 uint64_t ws_bytes, hipStream_t s);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of decode requests                        */
/* ---------------------------------------------------------------------- */

typedef struct {
  uint64_t mem_budget;         /* device bytes for outputs of admitted requests */
  uint32_t slots;              /* batches in flight at once (one HIP stream each), 1..16 */
  uint32_t max_batch;          /* requests per batch */
  uint32_t max_blocks;         /* blocks per batch (work-queue capacity) */
  uint32_t merge_variant;      /* merge kernel variant (see pivco_merge_variants) */
  uint64_t max_scratch_words;  /* rANS scratch words per batch */
  uint32_t keep_outputs;       /* 1: never recycle output space (for checking results) */
  uint32_t max_tiles;          /* 32Ki-symbol tiles of split blocks per batch (blocks of
                                  more than 64Ki symbols decode as tiles); 0 = 8192 */
} pivco_server_opts;

typedef struct {
  double arrival_s;            /* arrival time, seconds after run() starts */
  uint32_t id;                 /* registered stream */
  uint32_t reserved;
} pivco_request;

typedef struct {
  int32_t status;              /* pivco_status of this request */
  uint32_t reserved;
  void *d_out;                 /* where its bytes were decoded (inside the pool) */
  uint64_t n_out;
  double t_admit, t_done;      /* seconds after run() starts; latency = t_done - arrival */
} pivco_request_result;

typedef struct {
  double wall_s;
  uint64_t bytes_decoded;
  uint64_t peak_pool_bytes;
  uint64_t batches;
  uint64_t max_batch;
  uint64_t max_busy_slots;     /* most batches in flight at once (slots busy together) */
} pivco_server_stats;

typedef struct pivco_server pivco_server;

/* Creates the server: per slot a non-blocking stream, a device workspace and
 * pinned staging (allocated here, never on the request path). */
pivco_status pivco_server_create(const pivco_server_opts *o, pivco_server **out);
void pivco_server_destroy(pivco_server *sv);
/* Device bytes held by the slot workspaces. */
uint64_t pivco_server_workspace_bytes(const pivco_server *sv);
/* Registers a stream resident in device memory (16-byte aligned); reads its
 * header once (synchronous).  *id names it in requests. */
pivco_status pivco_server_register(pivco_server *sv, const void *d_stream, uint64_t len,
                                   uint32_t *id);
/* Replays the request trace (sorted by arrival) in real time: arrivals are
 * admitted FIFO while a slot is free and the output fits in the budget
 * (outputs are placed in d_pool, at most min(pool_bytes, mem_budget) bytes);
 * each admission round is one batched decode on a free slot, overlapping
 * with batches on other slots.  A request larger than the budget gets
 * PIVCO_E_BUDGET, and so does a request that does not fit in the pool while
 * no batch is in flight (with keep_outputs, output space is never released,
 * so requests after the pool has filled up fail this way).  Returns when
 * every request has completed or failed. */
pivco_status pivco_server_run(pivco_server *sv, const pivco_request *reqs, uint32_t n_req,
                              void *d_pool, uint64_t pool_bytes, pivco_request_result *res,
                              pivco_server_stats *stats);

const char *pivco_strerror(pivco_status st);

#ifdef __cplusplus
}
#endif
#endif
