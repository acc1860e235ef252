/*
 * qrng_ext.h -- C ABI of the MI355X (gfx950) block-wise two-source extractor.
 *
 * Operation (Li & Zhou, "Real-Time Seedless Post-Processing for Quantum
 * Random Number Generators"):
 *
 *   Two independent raw sample streams X and Y (b bits per sample, Sec. 3)
 *   are cut into consecutive blocks of n bits (Algorithm 1, equal blocks).
 *   Block l of X and block l of Y are each read as n_e = n/m elements of
 *   F_{2^m}, and the pair is mapped to the m-bit inner product
 *       Z^(l) = sum_{i<n_e} x_i * y_i          (Def. 3.2, Ext_IP^{n_e, m})
 *   in F_{2^m} (addition = bitwise XOR, Sec. 3.2).  The output stream is
 *   Z^(0) Z^(1) Z^(2) ... in block order (Thm. 3.6, Thm. 3.7).
 *
 * Conventions (the paper leaves them open; fixed here, identical for every
 * entry point):
 *   - F_{2^m} = GF(2)[t]/(P), polynomial basis: bit j of an element is the
 *     coefficient of t^j.  P is the lowest-weight irreducible polynomial of
 *     degree m, ties broken by the lexicographically smallest exponent tuple
 *     (trinomial t^m+t^a+1 with least a, else pentanomial
 *     t^m+t^a+t^b+t^c+1 with least a, then b, then c), unless the caller
 *     supplies other taps in ext_params.
 *   - bit r of a block is bit (r mod 8) of byte r/8 of the block (LSB first;
 *     for 8-bit samples a block is exactly n/8 consecutive samples, and the
 *     bytes are used as they are);
 *   - element i of a block is block bits [i*m, (i+1)*m);
 *   - block l of a stream is stream bytes [l*n/8, (l+1)*n/8);
 *   - output coefficient j of Z^(l) is output bit l*m + j, bytes LSB first
 *     (m/8 bytes per block pair, little-endian 32-bit words).
 *
 * Supported shapes on the GPU path: m a multiple of 8 (and of b), n a
 * multiple of m, and every non-leading exponent of P at most m/2 (the
 * conventional modulus qualifies for every such m from 8 to 8192).  Fields whose
 * degree is not a multiple of 32, or whose word count has an odd part above
 * 15, are computed in zero-padded slots; blocks and outputs may then sit at
 * any byte.  Everything else returns EXT_ENOTSUP.
 *
 * Errors: every call returns EXT_OK (0) or a negative ext_status; no call
 * aborts or throws.  A HIP failure is reported as EXT_EDEVICE and is sticky:
 * every later call on that context returns EXT_EDEVICE.
 *
 * Threading: one thread at a time per context (and per stream); distinct
 * contexts may be used concurrently.
 */
#ifndef QRNG_EXT_H
#define QRNG_EXT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ext_ctx ext_ctx;       /* opaque: shape, modulus, device buffers */
typedef struct ext_stream ext_stream; /* opaque: one (X, Y) channel pair */

enum ext_status {
    EXT_OK = 0,
    EXT_EINVAL = -1,  /* bad argument */
    EXT_ENOTSUP = -2, /* shape or modulus outside what the GPU path supports */
    EXT_ENOMEM = -3,  /* host or device allocation failed */
    EXT_EAGAIN = -4,  /* admission: the stream's device buffer is full, poll and retry */
    EXT_EDEVICE = -5, /* HIP runtime error (sticky on the context) */
    EXT_ECLOSED = -6  /* stream already closed */
};

enum ext_mem_kind {
    EXT_MEM_HOST = 0,  /* pointers passed to ext_extract/ext_submit/ext_poll are host memory */
    EXT_MEM_DEVICE = 1 /* they are device memory of the context's device */
};

typedef struct {
    uint32_t sample_bits;       /* b, bits per raw sample; 0 means 8.  m % b must be 0
                                   (the paper makes m a multiple of b, Algorithm 1). */
    uint32_t n_taps;            /* 0: conventional modulus; 1: trinomial; 3: pentanomial */
    uint32_t taps[3];           /* non-leading nonzero exponents of P, any order
                                   (P = t^m + sum t^taps[k] + 1); checked irreducible */
    uint32_t mem_kind;          /* enum ext_mem_kind */
    void *hip_stream;           /* hipStream_t to run on (NULL is the null stream) */
    uint32_t use_hip_stream;    /* 1: run on hip_stream; 0: the library creates a stream */
    uint64_t device_bytes_cap;  /* per stream: cap on pending input bytes held on the
                                   device (admission); 0 means 256 MiB */
    int32_t device;             /* HIP device ordinal; -1 means the current device */
    /* launch-plan knobs, 0 = the planner's choice (the autotuner sets them) */
    uint32_t base_bits;         /* Karatsuba base-product size in bits (multiple of 32) */
    uint32_t groups;            /* element groups per work item (divides n/m) */
    uint32_t pairs_per_group;   /* block pairs per work-group */
    uint32_t autotune;          /* 1: time the candidate plans on the device at create
                                   time and keep the fastest (cached per shape) */
    uint32_t threads;           /* work-group size, 0 = 256; 1024 shortens the critical
                                   path of shapes with more than 256 items per pair */
    uint32_t kernel;            /* plain and streaming forms: EXT_KERNEL_AUTO (default),
                                   EXT_KERNEL_WORD (word-level Karatsuba kernel) or
                                   EXT_KERNEL_BITSLICE (32 pairs per work-group bit-sliced
                                   across pairs; fields of at most 128 bits, else
                                   EXT_ENOTSUP).  Both give the same bytes.  AUTO takes
                                   the bit-sliced kernel for fields of 16 to 128 bits
                                   that 16 divides with at least 30 elements per block
                                   (where it measured faster), or, with autotune set,
                                   whichever of the two times faster for the shape.
                                   The batched, served and growing forms run the
                                   word-level kernel: they answer EXT_KERNEL_BITSLICE
                                   with EXT_ENOTSUP */
    uint32_t reserved[2];
} ext_params;
enum { EXT_KERNEL_AUTO = 0, EXT_KERNEL_WORD = 1, EXT_KERNEL_BITSLICE = 2 };

/* Fill *p with defaults (b = 8, conventional modulus, host memory, a stream
 * of the library's own, 256 MiB cap, current device). */
void ext_params_init(ext_params *p);

/*
 * Create a context for blocks of n_bits bits and m_bits output bits per
 * block pair (n_e = n_bits / m_bits elements of F_{2^m}, Def. 3.2).
 * *out is owned by the caller and released by ext_destroy.
 * EXT_EINVAL: n_bits or m_bits zero, n_bits % m_bits, m % b, bad taps or a
 *             reducible P.  EXT_ENOTSUP: see "Supported shapes" above.
 */
int ext_create(uint64_t n_bits, uint32_t m_bits, const ext_params *p, ext_ctx **out);

/* Release the context and every stream still open on it (waits for queued
 * GPU work first).  NULL is accepted. */
int ext_destroy(ext_ctx *c);

/* Exponents of the context's modulus P in decreasing order (m first, 0
 * last).  cap >= 5 always suffices; *n receives the count. */
int ext_get_modulus(const ext_ctx *c, uint32_t *exps, uint32_t cap, uint32_t *n);

/* The conventional modulus of degree m (see Conventions) without creating a
 * context: same output format as ext_get_modulus.  The library's table holds
 * every multiple of 8 up to 8192 (and 16384); other degrees up to 32768 are
 * searched at first use (on up to 16 host threads; about a second at 10000
 * bits, minutes at 32768) and cached; EXT_ENOTSUP above 32768. */
int ext_default_modulus(uint32_t m_bits, uint32_t *exps, uint32_t cap, uint32_t *n);

/* 1 if t^m + sum t^taps + 1 is irreducible over GF(2), 0 if not, <0 on a
 * bad argument.  Rabin's test. */
int ext_is_irreducible(uint32_t m_bits, const uint32_t *taps, uint32_t n_taps);

/*
 * Growing blocks (Algorithm 2): block l (from 0) holds q_l * n_e bits of each
 * source, right after block l-1, with q_l = q1 + l * delta_steps * b (b =
 * p->sample_bits), and yields Ext_IP^{n_e, q_l} of the two blocks, q_l bits,
 * outputs concatenated (block l's q_l/8 bytes right after block l-1's).
 * delta_steps = 0 is Algorithm 1.  Each degree uses the conventional modulus
 * (p->n_taps must be 0); q1 and delta_steps * b must be multiples of 8, and
 * q1 a multiple of b.
 */
typedef struct ext_growing ext_growing;
int ext_growing_create(uint32_t n_e, uint32_t q1, uint32_t delta_steps, const ext_params *p,
                       ext_growing **out);
/* How many whole blocks the first n_bytes of each source hold, and their
 * input bytes (per source) and output bytes (any pointer may be NULL). */
int ext_growing_blocks(const ext_growing *g, uint64_t n_bytes, uint64_t *k_blocks,
                       uint64_t *in_bytes, uint64_t *out_bytes);
/* Blocks 0 .. k-1 of the streams x and y (n_bytes each, from block 0; k =
 * the whole blocks they hold, at most max_blocks) into out (out_cap bytes, at
 * least the k blocks' output bytes, else EXT_EINVAL); *n_blocks = k.  Memory
 * kind and stream as for ext_extract; returns after the outputs are written.
 * EXT_ENOTSUP if some q_l has no conventional modulus in reach (above 32768
 * bits; see ext_default_modulus) or no launch plan. */
int ext_growing_extract(ext_growing *g, const void *x, const void *y, uint64_t n_bytes,
                        uint64_t max_blocks, void *out, uint64_t out_cap, uint64_t *n_blocks);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ext_growing_extract on device memory, with the same arguments, results
 * and errors, that allocates nothing.  Its launch tables and queue heads
 * live in a static device array of the library (about 0.7 MiB, one copy per
 * GPU, held until the process ends; its address on each GPU is looked up
 * when an ext_growing is first created there) instead of buffers the handle
 * allocates.  The queue heads are cleared by every call.
 *   - the handle must have been created with mem_kind = EXT_MEM_DEVICE, else
 *     EXT_EINVAL;
 *   - at most EXT_NOALLOC_MAX_BLOCKS blocks per call: a call whose k (the
 *     whole blocks in n_bytes, capped by max_blocks) is larger returns
 *     EXT_ENOMEM and does nothing;
 *   - EXT_EDEVICE if the array's address could not be looked up.
 * Every call on a GPU, from any handle, uses that GPU's one array: calls
 * that overlap on one GPU race and must be serialised by the caller (this
 * call returns after its outputs are written, so one thread at a time per
 * GPU suffices).
 */
/*
 * Online form of Algorithm 2 (Sec. 3.3, Ext_bs^neq on sources of unbounded
 * length): X and Y arrive in chunks of any length, the two sides
 * independently.  The stream carries Algorithm 2's state from call to call --
 * the next block l (from 0), its degree q_l = q1 + l * delta_steps * b, and i,
 * the bytes per source that blocks 0 .. l-1 took -- and keeps the bytes of
 * the block still incomplete in device memory.  Block l is launched as soon
 * as both sources hold its q_l * n_e / 8 bytes; its q_l / 8 output bytes come
 * back from ext_growing_poll in block order, each exactly once, so that after
 * k blocks the caller holds Z^(0) Z^(1) ... Z^(k-1), m_k bits (Thm. 3.6).
 * Memory kind, HIP stream and device come from g; one thread at a time per
 * handle (streams of one handle share its GPU streams).
 */
typedef struct ext_growing_stream ext_growing_stream;
/* Open a stream on g in state (l, q_l, i) = (0, q1, 0).  Released by
 * ext_growing_close (or ext_growing_destroy of g). */
int ext_growing_open(ext_growing *g, ext_growing_stream **out);
/* Append x_len bytes to X and y_len bytes to Y (either may be 0): the next
 * samples of each source.  Host data are copied before the call returns;
 * device data are read in stream order and borrowed until that work is done.
 * Launches every block the chunk completes.  Nothing is consumed when the
 * call returns
 *   EXT_EAGAIN  if either side would hold more pending bytes than its limit
 *               -- device_bytes_cap, lowered so that their outputs fit in
 *               half of the stream's output ring (1 to 64 MiB), and never
 *               below two blocks of the next degree -- or the outputs of the
 *               completed blocks would not fit beside the unpolled ones:
 *               poll (or feed the other side), then submit again;
 *   EXT_ENOTSUP if a completed block's degree has no conventional modulus in
 *               reach (above 32768 bits, or beyond the built-in table of the
 *               multiples of 8 up to 8192 and a search, run at first use,
 *               that fails) or no launch plan.
 * *blocks_launched (may be NULL): blocks launched so far. */
int ext_growing_submit(ext_growing_stream *s, const void *x, size_t x_len, const void *y,
                       size_t y_len, uint64_t *blocks_launched);
/* Non-blocking: copy finished outputs into out (host or device memory per
 * mem_kind), whole blocks only, in block order, at most out_cap bytes;
 * *out_len: bytes written; *blocks_done (may be NULL): blocks returned so far
 * over the stream's life.  Device memory on the caller's HIP stream
 * (use_hip_stream): the copies are queued on that stream and complete in its
 * order; otherwise they are complete when the call returns. */
int ext_growing_poll(ext_growing_stream *s, void *out, size_t out_cap, size_t *out_len,
                     uint64_t *blocks_done);
/* As ext_growing_poll, but first waits for every launched block, and
 * returns after its copies are complete. */
int ext_growing_drain(ext_growing_stream *s, void *out, size_t out_cap, size_t *out_len,
                      uint64_t *blocks_done);
/* Algorithm 2's state: the next block l, its degree q_l, and the bytes per
 * source taken by blocks 0 .. l-1 (any pointer may be NULL). */
int ext_growing_state(const ext_growing_stream *s, uint64_t *next_block, uint64_t *next_q,
                      uint64_t *consumed_bytes);
/* Close: the incomplete block is dropped (Algorithm 2 outputs whole blocks
 * only) and its size, the larger side's pending bytes in bits, reported in
 * *dropped_bits (may be NULL); outputs not yet polled are discarded. */
int ext_growing_close(ext_growing_stream *s, uint64_t *dropped_bits);

enum { EXT_NOALLOC_MAX_BLOCKS = 4096 };
int ext_growing_extract_noalloc(ext_growing *g, const void *x, const void *y, uint64_t n_bytes,
                                uint64_t max_blocks, void *out, uint64_t out_cap,
                                uint64_t *n_blocks);
int ext_growing_destroy(ext_growing *g);

/*
 * Parameters and security bounds (host only, no GPU work).
 *
 * ext_choose_params: Algorithm 1's rule for two (b, N, delta) forward block
 * sources and a total error eps: n_e = ceil(24 / (2 delta - 1)) elements per
 * block (integer arithmetic on delta = delta_num / delta_den, which must lie
 * in (1/2, 1]) and q = b * ceil(log2(N / (eps n_e)) / b) bits per element
 * (double precision; N given as log2 of the number of b-bit samples per source,
 * eps as log2 of the error, which must be negative).  EXT_EINVAL when the
 * inputs are outside those ranges or q would not be positive.
 */
int ext_choose_params(uint32_t sample_bits, uint64_t delta_num, uint64_t delta_den,
                      double log2_n_samples, double log2_eps, uint32_t *n_e, uint32_t *q);
/* Theorem 3.3: log2 of sqrt(3) * 2^(-1/4 - (delta/4 - 1/8) q n_e + 2q), the
 * distance from uniform of one block's output for sources of min-entropy rate
 * delta (a value >= 0 means the bound says nothing).  NaN on a bad argument. */
double ext_block_error_log2(uint32_t n_e, uint32_t q, double delta);
/* Theorem 3.6, for Algorithm 2 with q_l = q1 + (l-1) * delta_steps * b
 * (delta_steps = 0 is Algorithm 1): *log2_sum = log2 of the sum of the k
 * per-block bounds (a geometric series, evaluated in closed form), and
 * *log2_closed = log2 of sqrt(3) 2^(-1/4 - q1) / (1 - 2^(-delta_steps b)), the
 * bound on the whole infinite output (+inf when delta_steps = 0).  Either
 * pointer may be NULL. */
int ext_stream_error_log2(uint32_t n_e, uint32_t q1, uint32_t delta_steps, uint32_t sample_bits,
                          double delta, uint64_t k, double *log2_sum, double *log2_closed);
/* Theorem 3.6: m_k = k q1 + k (k-1) delta_steps b / 2 output bits of the
 * first k blocks; EXT_EINVAL if it does not fit in 64 bits. */
int ext_output_bits(uint32_t q1, uint32_t delta_steps, uint32_t sample_bits, uint64_t k,
                    uint64_t *m_k);

/*
 * Plain form (Algorithm 1 over n_pairs whole block pairs).
 *   x, y : n_pairs * n/8 bytes each (block l at byte offset l*n/8),
 *          4-byte aligned; 16-byte aligned device memory when m is 128
 *          or 256 (those shapes read their operands with 16-byte loads)
 *   out  : n_pairs * m/8 bytes, 4-byte aligned
 * EXT_MEM_DEVICE: x, y, out are device pointers; the work is queued on the
 *   context's stream and the call returns at once (synchronize the stream,
 *   or call ext_sync, before reading out).  The buffers are borrowed until
 *   that work completes.
 * EXT_MEM_HOST: the call copies x and y to the device, runs, copies the
 *   result to out and returns when out is complete.
 * n_pairs == 0 is a no-op.
 */
int ext_extract(ext_ctx *c, const void *x, const void *y, uint64_t n_pairs, void *out);

/* Wait for every piece of work queued by this context. */
int ext_sync(ext_ctx *c);

/*
 * Streaming form: Algorithm 1 run online.  The paper's sources are unbounded
 * sample streams X and Y (Sec. 3); block l is the restriction X_{I_l} of a
 * source to the l-th run of n/b consecutive samples (Algorithm 1's loop over
 * the index sets I_l), and the output is the concatenation Z^(0) Z^(1) ... of
 * the per-block results (Thm. 3.6, Thm. 3.7).  A stream is one (X, Y) channel
 * pair fed in chunks of any length, the two sides independently; the partial
 * block still waiting for data stays on the device.  Block l is computed as
 * soon as both sides hold (l+1)*n/8 bytes; outputs come back from ext_poll
 * strictly in block order, each exactly once.
 */

/*
 * Open a stream on context c.  n_bits and m_bits give the stream's own block
 * length and output size; 0 takes the context's.  A stream whose shape
 * differs from the context's uses the context's modulus when m_bits equals
 * the context's m, else the conventional modulus of degree m_bits (see
 * Conventions), and the planner's default launch plan for its shape; its
 * kernel follows the context's ext_params.kernel.  The shape rules are those
 * of ext_create (EXT_EINVAL, EXT_ENOTSUP).  Memory kind, stream, device and
 * the per-stream device_bytes_cap come from the context.  *out is released
 * by ext_stream_close (or ext_destroy of c).
 */
int ext_stream_open(ext_ctx *c, uint64_t n_bits, uint32_t m_bits, ext_stream **out);

/*
 * Append x_len bytes to X and y_len bytes to Y (either may be 0): the next
 * samples of each source, in order.  The data are copied before the call
 * returns (host memory) or read in stream order on the context's stream
 * (device memory, borrowed until that work is done).  Launches the
 * extraction of every block pair I_l completed by this chunk.
 * EXT_EAGAIN: the bytes held on the device would exceed device_bytes_cap;
 * nothing was consumed -- poll, then submit again.
 * *seq_out (may be NULL) receives the number of block pairs launched so far.
 */
int ext_submit(ext_stream *s, const void *x, size_t x_len, const void *y, size_t y_len,
               uint64_t *seq_out);

/*
 * Non-blocking: copy finished outputs Z^(l), in block order (the
 * concatenation of Thm. 3.6/3.7), into out (host or device memory per
 * mem_kind), at most out_cap bytes and only whole blocks (m/8 bytes each).
 * *out_len receives the bytes written; *blocks_done (may be NULL) the number
 * of blocks returned so far over the stream's life.
 */
int ext_poll(ext_stream *s, void *out, size_t out_cap, size_t *out_len, uint64_t *blocks_done);

/* Blocking variant of ext_poll: waits until every launched block is done,
 * then copies as ext_poll does. */
int ext_drain(ext_stream *s, void *out, size_t out_cap, size_t *out_len, uint64_t *blocks_done);

/*
 * Close the stream: the trailing partial block (fewer than n bits on either
 * side; Algorithm 1 consumes whole blocks only) is dropped and its size, max
 * over the two sides, is reported in *dropped_bits (may be NULL).  Outputs
 * not yet polled are discarded.  The handle is freed; using it afterwards is
 * undefined.
 */
int ext_stream_close(ext_stream *s, uint64_t *dropped_bits);

/*
 * Batched form: many independent stream pairs, each with its own block
 * length n and output size m, computed by ONE persistent launch per base
 * size that drains a device work queue of tiles (a stream's next few block
 * pairs), the launches captured once in a hipGraph and replayed by
 * ext_batch_run.  Every pointer is device memory of the batch's device and
 * is borrowed for the life of the batch (the graph holds the addresses; the
 * contents may change between runs).  Each item uses the conventional
 * modulus of its m; the shape rules are those of ext_create.
 */
typedef struct ext_batch ext_batch;
typedef struct {
    uint64_t n_bits;     /* block length n of this stream pair */
    uint32_t m_bits;     /* output bits per block pair */
    uint32_t reserved;
    const void *x, *y;   /* n_pairs * n/8 bytes each */
    void *out;           /* n_pairs * m/8 bytes */
    uint64_t n_pairs;
} ext_batch_item;

/* Plan every item (ext_params.autotune = 1 times candidate plans per shape
 * on the device first), build the tile queue and capture the launches.
 * p may be NULL; p->n_taps must be 0.  Uses p->hip_stream when
 * use_hip_stream is set and the handle is not the null stream, else a stream
 * of its own. */
int ext_batch_create(const ext_batch_item *items, uint32_t n_items, const ext_params *p,
                     ext_batch **out);
/* Queue one pass over every item (asynchronous, on the batch's stream). */
int ext_batch_run(ext_batch *b);
/* Wait for the batch's stream. */
int ext_batch_sync(ext_batch *b);
/* One-line JSON: streams, tiles, pairs, launches (base size, tiles, grid). */
int ext_batch_describe(const ext_batch *b, char *buf, size_t cap);
/* Wait for queued work, then free.  NULL is accepted. */
int ext_batch_destroy(ext_batch *b);

/*
 * Served form: continuous batching of many generator channels.  Each channel
 * is an (X, Y) pair of raw sample streams with its own block length n and
 * output size m (conventional modulus).  Chunks of any length arrive through
 * ext_server_submit (host memory, copied before the call returns); a
 * scheduler thread inside the server repeatedly takes everything that
 * arrived, moves it to the channels' device rings and computes every block
 * pair completed so far on every channel in one persistent launch per base
 * size, while earlier cycles may still be on the GPU (at most max_inflight).
 * Outputs come back per channel, in block order, exactly once.
 * Admission: a channel is admitted by free device memory -- ext_server_open
 * allocates the channel's two device rings only if they fit in the device's
 * free memory (hipMemGetInfo) less device_reserve_bytes, and within
 * rings_bytes_cap over all open channels, else returns EXT_EAGAIN with
 * nothing allocated (retry once channels have closed).  Every other device
 * buffer is allocated at create time, so a submission never needs more
 * device memory: a channel holds at most its ring's worth of blocks between
 * received and polled, and a cycle takes at most stage_bytes of input and
 * returns at most outbox_bytes of output; beyond that ext_server_submit
 * returns EXT_EAGAIN and consumes nothing.  All calls are thread-safe.
 */
typedef struct ext_server ext_server;
typedef struct {
    uint32_t max_channels;  /* channel slots (default 256) */
    uint32_t ring_blocks;   /* device ring per channel side, in blocks; 0 = sized by
                               ring_bytes (default 0) */
    uint64_t stage_bytes;   /* input bytes one cycle can take (default 64 MiB) */
    uint64_t outbox_bytes;  /* output bytes one cycle can return (default 32 MiB) */
    uint32_t max_tiles;     /* work-group tiles per cycle (default 131072) */
    uint32_t max_descs;     /* copy ranges per cycle (default 65536) */
    uint32_t poll_us;       /* scheduler re-check period while a cycle runs; 0 or 1 = keep
                               checking (yielding the CPU between checks; default 0) */
    uint32_t wg_per_cu;     /* at most this many persistent work-groups per CU in a
                               cycle's launch (enforced through the LDS request when the
                               device allows it); 0 = as many as fit (default 0) */
    uint64_t ring_bytes;    /* when ring_blocks == 0: ring per channel side in bytes, rounded
                               down to whole blocks, at least 128 blocks (default 4 MiB) */
    uint32_t max_inflight;  /* cycles on the GPU at once, 1..3; a cycle's staging runs on
                               its own stream and may overlap the previous cycle's
                               extraction, and a new cycle starts only once the previous
                               one is staged (default 2) */
    uint32_t split_pairs;   /* 1: plan channels for latency: one base product per lane
                               item, and a pair with more items than a work-group has
                               lanes is split over several work-groups whose partial sums
                               a combine step adds and reduces; 0: whole pairs per
                               work-group, with the plain form's plan (default 1) */
    uint32_t timing;        /* 1: time every cycle's phases on the GPU with events (the
                               gpu_ns, stage_ns and extract_ns stats); default 0 */
    uint32_t reserved;
    uint64_t device_reserve_bytes; /* admission: device memory a channel open must leave
                                      free (default 1 GiB) */
    uint64_t rings_bytes_cap;      /* admission: device bytes the rings of all open
                                      channels may hold together; 0 = no cap beyond free
                                      memory (default 0) */
} ext_server_config;
typedef struct {
    uint64_t cycles, tiles, pairs, bytes_in;
    uint64_t eagain_ring;   /* submissions refused: channel ring full */
    uint64_t eagain_stage;  /* submissions refused: cycle staging full */
    uint64_t gpu_busy_ns;   /* sum over cycles of launch-to-harvest time */
    uint64_t split_pairs;   /* pairs computed as slices over several work-groups */
    uint64_t build_ns;      /* host time spent building cycles (tiles, metadata) */
    uint64_t launch_ns;     /* host time spent queueing cycles' kernels and events */
    uint64_t max_cycle_ns;  /* longest launch-to-harvest time of a cycle */
    uint64_t gpu_ns;        /* with timing: sum over cycles of the GPU time from the first
                               kernel's start to the end of the last */
    uint64_t stage_ns;      /* of which: staging the cycle's input and metadata */
    uint64_t extract_ns;    /* of which: the extraction launches (the rest: combine) */
    uint64_t eagain_mem;    /* channel opens refused: rings beyond free device memory less
                               the reserve, or beyond rings_bytes_cap */
    uint64_t rings_bytes;   /* device bytes the open channels' rings hold now */
    uint64_t free_bytes;    /* the device's free memory at the last channel open */
} ext_server_stats;

void ext_server_config_init(ext_server_config *c);
/* cfg and p may be NULL (defaults); p->n_taps must be 0; p->autotune,
 * base_bits, groups, pairs_per_group, device and hip_stream apply. */
int ext_server_create(const ext_server_config *cfg, const ext_params *p, ext_server **out);
/* Open a channel; *channel receives its index.  EXT_EAGAIN: no free slot,
 * or its rings do not fit in free device memory less the reserve or under
 * rings_bytes_cap (nothing allocated). */
int ext_server_open(ext_server *s, uint64_t n_bits, uint32_t m_bits, uint32_t *channel);
int ext_server_submit(ext_server *s, uint32_t channel, const void *x, size_t x_len,
                      const void *y, size_t y_len);
/* Non-blocking.  Copies finished outputs (whole blocks, block order) into
 * host memory out; ready_ns (may be NULL, room for out_cap/(m/8) entries)
 * receives for each returned block the steady-clock time (ns) at which the
 * server saw it finish; *blocks_done the blocks returned so far. */
int ext_server_poll(ext_server *s, uint32_t channel, void *out, size_t out_cap, size_t *out_len,
                    uint64_t *ready_ns, uint64_t *blocks_done);
/* Wait up to timeout_us for channels with output not yet polled; writes up
 * to cap channel indices to chans and their count to *n (0 on timeout). */
int ext_server_ready(ext_server *s, uint32_t *chans, uint32_t cap, uint32_t *n,
                     uint32_t timeout_us);
/* Close a channel after its launched pairs finish; the trailing partial
 * block and any unpolled output are dropped (*dropped_bits: input bits not
 * part of a complete pair, larger side). */
int ext_server_close(ext_server *s, uint32_t channel, uint64_t *dropped_bits);
int ext_server_stats_get(ext_server *s, ext_server_stats *out);
/* Stop the scheduler after the cycles in flight, then free everything. */
int ext_server_destroy(ext_server *s);

/*
 * Load generator for the served form: replays Poisson chunk arrivals on many
 * channels in real time against either the server (EXT_SIM_SERVED) or the
 * plain streaming form with one ext_stream and one launch per arriving chunk
 * per channel (EXT_SIM_PLAIN), and measures per-block latency from the
 * scheduled arrival of the chunk that completes a block to the moment a
 * poll returns its output.
 */
enum { EXT_SIM_SERVED = 0, EXT_SIM_PLAIN = 1 };
typedef struct {
    uint32_t n_channels;
    uint32_t mode;                  /* EXT_SIM_SERVED or EXT_SIM_PLAIN */
    const uint64_t *n_bits;         /* per channel */
    const uint32_t *m_bits;         /* per channel */
    const uint8_t *const *pool_x;   /* per channel: source bytes, read cyclically */
    const uint8_t *const *pool_y;
    const uint64_t *pool_bytes;     /* per channel: pool length, a multiple of n/8 */
    double raw_bytes_per_s;         /* aggregate X+Y input rate, split evenly over channels */
    uint32_t min_chunk_blocks, max_chunk_blocks;  /* chunk = k blocks of X and of Y, k uniform */
    double warmup_s, duration_s;    /* latency counted for arrivals in [warmup, warmup+duration) */
    double grace_s;                 /* wait after the last arrival for outstanding blocks */
    double max_lag_s;               /* stop submitting once this far behind schedule (0 = never);
                                       the chunks left count as missing */
    uint64_t seed;
    uint32_t producer_threads;      /* submitting threads (channels split among them); 0 = 4 */
    uint32_t reserved0;
    uint8_t *const *capture;        /* optional per channel: every output byte, in order */
    const uint64_t *capture_cap;    /* per channel capacity of capture */
    const ext_server_config *server_cfg;  /* served mode; NULL = defaults */
    const ext_params *params;       /* NULL = defaults */
} ext_sim_config;
typedef struct {
    double window_s;                /* measurement window length */
    double out_gbps, in_gbps;       /* bits of blocks arrived in the window and returned, / window */
    double offered_in_gbps;         /* raw bits scheduled in the window / window */
    double lat_p50_us, lat_p99_us, lat_max_us, lat_mean_us;
    uint64_t blocks_measured;       /* blocks arrived in the window */
    uint64_t blocks_missing;        /* of those, not returned before the grace time ran out */
    uint64_t chunks, eagain;
    double max_submit_lag_us;       /* worst lateness of a submission behind its schedule */
    uint64_t cycles;                /* served mode: scheduler cycles */
    uint64_t eagain_ring;           /* served mode: refusals because a channel ring was full */
    uint64_t eagain_stage;          /* served mode: refusals because a cycle was full */
    double mean_cycle_us;           /* served mode: mean launch-to-harvest time of a cycle */
    double submit_lag_p99_us;       /* chunks arrived in the window: p99 of the time from the
                                       scheduled arrival to the return of their submission */
    double service_p50_us, service_p99_us;  /* blocks arrived in the window: from the return
                                       of the submission that completed them to the poll */
    double ready_p50_us, ready_p99_us;  /* served mode, same blocks: from that return to the
                                       moment the server had their output in host memory */
    double mean_build_us;           /* served mode: host time to build a cycle, mean */
    double mean_launch_us;          /* served mode: host time to queue a cycle, mean */
    double max_cycle_us;            /* served mode: longest launch-to-harvest time */
    double mean_gpu_us;             /* served mode: GPU time of a cycle, mean */
    double mean_tiles;              /* served mode: work-group tiles per cycle, mean */
    double mean_stage_us, mean_extract_us;  /* served mode: parts of mean_gpu_us */
    uint64_t rings_bytes;           /* served mode: device bytes the channels' rings held
                                       (admitted against free device memory) */
    uint64_t free_bytes;            /* served mode: device free memory at the last open */
    uint64_t eagain_mem;            /* served mode: channel opens refused for memory */
} ext_sim_result;
/* capture_len (may be NULL): per channel, bytes written to capture. */
int ext_serve_simulate(const ext_sim_config *cfg, ext_sim_result *res, uint64_t *capture_len);

/* Write a one-line JSON description of the context's launch plan (base
 * product size, Karatsuba levels, work-group shape) into buf (1024 bytes
 * suffice).  A word-level context planned without fixed knobs also has
 * latency plans (one element per lane item; half the base size, and smaller
 * ones while a pair's n_e * 3^levels items fit in one work-group's lanes)
 * that plain and streaming launches take when the default plan would give
 * fewer work-groups than the GPU has compute units: the smallest base whose
 * launch stays within two work-groups per compute unit, else the half-size
 * one.  "small_launch" describes the smallest and lists every base. */
int ext_describe(const ext_ctx *c, char *buf, size_t cap);

/* Diagnostic: the device's measured issue rate of the extraction kernel's
 * AND-XOR (v_bitop3_b32), in 32-bit lane operations per second, from a
 * ~10 ms probe kernel of independent chains on every CU (device < 0: the
 * current device).  Used to state a kernel's VALU issue utilisation against
 * what the chip delivers at that moment. */
int ext_probe_valu_rate(int device, double *lane_ops_per_s);

/* Static description of a status code. */
const char *ext_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* QRNG_EXT_H */
