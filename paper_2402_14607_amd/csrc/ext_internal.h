// ext_internal.h -- shapes and launchers shared by the C ABI (ext_api.cpp)
// and the gfx950 kernels (ext_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qext {

constexpr int kThreads = 256;           // default work-group size of the extraction kernel
constexpr int kMaxThreads = 1024;       // largest work-group size of the extraction kernels
constexpr int kMaxBaseWords = 16;       // largest base-product size, 32-bit words
constexpr uint32_t kMaxLdsBytes = 32768;
constexpr uint32_t kPadRegs = 16;       // slot words per lane in padded staging
constexpr uint32_t kPadSlack = 8;       // words after each staged area of a padded shape

// Launch shape of one (n, m, P) configuration; computed on the host by
// plan_shape() and passed to the kernel by value.
struct ExtShape {
    uint32_t q;        // m, field degree = output bits per block pair
    uint32_t qw;       // ceil(q / 32), words per element (padded when q % 32 != 0)
    uint32_t n_e;      // elements per block (n / m)
    uint32_t nw;       // qw * n_e, words per block (in its padded LDS layout if padded)
    uint32_t bw;       // base-product size in words (B = 32*bw bits)
    uint32_t levels;   // Karatsuba levels L, q = B * 2^L
    uint32_t np;       // 3^L sub-products per element product
    uint32_t ppw;      // block pairs per work-group
    uint32_t groups;   // element groups per (pair, sub-product) work item
    uint32_t epg;      // elements per group (n_e / groups)
    uint32_t stage;    // 1: the work-group's input blocks are staged in LDS
    uint32_t n_taps;   // 1 (trinomial) or 3 (pentanomial)
    uint32_t taps[3];  // non-leading nonzero exponents of P, each at most q/2
    uint32_t dn;       // words of the second reduction pass, ceil((max tap - 1)/32)
    uint32_t lds_words;
    uint32_t align;    // required byte alignment of x and y (16 when operands are
                       // read from HBM with 16-byte loads, else 4)
    uint32_t threads;  // work-group size (a multiple of 64, at most kMaxThreads)
    uint32_t padded;   // 1: q is not a multiple of 32; elements are re-laid out
                       // in LDS as qw-word slots (qw = ceil(q/32)) and outputs
                       // stored as bytes
    uint32_t qbytes;   // q / 8, output bytes per pair
    uint32_t nbytes;   // n / 8, bytes per block
};

// Tuning choices for one shape; 0 in a field means "planner's choice".
struct PlanKnobs {
    uint32_t base_words;  // base-product size in 32-bit words (1..16)
    uint32_t groups;      // element groups per work item (divides n_e)
    uint32_t ppw;         // block pairs per work-group
    uint32_t threads;     // work-group size (256 or 1024)
    uint32_t padded;      // 1: use the padded layout even when q is a multiple of 32
                          // (byte-granular blocks and outputs)
    uint32_t max_odd;     // largest odd part of the (padded) words per element, which
                          // bounds the base product (0: 15)
};

// LDS bytes one work-group of shape s takes in the plain and batched kernels:
// lds_words, plus, for unpadded shapes (whose pairs the kernels lay out
// rank-major at padded strides), 4 words per staged block and side and 1 per
// sum, for each pair.
inline uint32_t group_lds_bytes(const ExtShape& s) {
    const uint32_t pad = s.padded ? 0u : s.ppw * (1u + (s.stage ? 8u : 0u));
    return (s.lds_words + pad) * 4u;
}

// Fills *s for q, n_e and the taps; returns false if the shape is outside
// what the kernel supports.
bool plan_shape(uint32_t q, uint32_t n_e, const uint32_t* taps, uint32_t n_taps,
                const PlanKnobs& knobs, ExtShape* s);

// One stream of a batch, as the batched kernel reads it from device memory:
// blocks shape.nbytes apart in x and y, outputs shape.qbytes apart in out.
struct BatchStream {
    const uint8_t* x;
    const uint8_t* y;
    uint8_t* out;
    uint64_t n_pairs;
    ExtShape shape;
};

// One work-group's worth of a batch: npw consecutive pairs of a stream,
// whose blocks start at pair slot in_pair0 of the stream's x and y, and
// whose outputs go to byte out_off of the stream's out.  When n_items is
// nonzero the tile is one slice of the single pair in_pair0 -- its items
// [item0, item0 + n_items) in element-major order, or for a padded shape its
// elements [item0, item0 + n_items) -- whose partial unreduced sum goes to
// word out_off of the launch's part buffer instead.
struct BatchTile {
    uint32_t stream;
    uint32_t npw;
    uint64_t in_pair0;
    uint64_t out_off;
    uint32_t item0;
    uint32_t n_items;
};

// One sliced pair to finish: XOR n_parts consecutive parts (2qw words each)
// starting at word part_word0 of the part buffer, reduce, and store the
// output at byte out_byte0 of the stream's out (a multiple of 4 unless the
// shape is padded).
struct CombineJob {
    uint32_t stream;
    uint32_t n_parts;
    uint64_t part_word0;
    uint64_t out_byte0;
};

// Queue the extraction of n_pairs consecutive block pairs on `stream`.
// x, y: device, n_pairs*nbytes bytes each; out: device, n_pairs*qbytes bytes
// (4-byte aligned unless the shape is padded).
hipError_t launch_extract(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                          uint64_t n_pairs, hipStream_t stream);

// Queue the queue-head reset and one persistent launch of `grid` work-groups
// of `threads` lanes over n_tiles tiles (all streams of the launch share base
// size bw, work-group size and whether their shape is padded).
// streams, tiles, head: device memory.
hipError_t launch_batch(uint32_t bw, uint32_t threads, bool padded, const BatchStream* streams,
                        const BatchTile* tiles, uint32_t n_tiles, uint32_t* head, uint32_t grid,
                        uint32_t lds_bytes, hipStream_t stream);

// Autotuner: time the candidate plans of (q, n_e, taps) on `stream` and
// return the fastest as knobs (cached per device and shape).
hipError_t autotune_shape(uint32_t q, uint32_t n_e, const uint32_t* taps, uint32_t n_taps,
                          hipStream_t stream, PlanKnobs* best, float* best_ms);

// Autotuned choice between the word-level kernel (its best plan) and the
// bit-sliced kernel for a shape the latter applies to; cached per device.
hipError_t choose_kernel(const ExtShape& bitslice_shape, hipStream_t stream, bool* use_bitslice);

// One byte range to move from a staging buffer into a device ring.
struct ScatterDesc {
    uint64_t src_off;  // byte offset in the staging buffer
    uint8_t* dst;      // device destination
    uint32_t len;      // bytes
    uint32_t pad;
};

// Queue a served cycle's staging kernel: copy every descriptor's range from
// src (the host's pinned staging area, read over the bus) into its ring, copy
// meta_bytes (a multiple of 16) from meta_src (pinned) to meta_dst (device),
// and clear n_heads queue heads.
hipError_t launch_stage(const uint8_t* src, const ScatterDesc* descs, uint32_t n_descs,
                        const void* meta_src, void* meta_dst, uint32_t meta_bytes, uint32_t* heads,
                        uint32_t n_heads, hipStream_t stream);

// Up to kMaxCopySegs byte ranges to copy on the device (sources in device
// memory or in pinned, coherent host memory; ranges neither overlap nor
// alias another segment's destination), passed to the kernel by value.
constexpr uint32_t kMaxCopySegs = 4;
struct CopySeg {
    const uint8_t* src;
    uint8_t* dst;
    uint64_t len;
};
struct CopySegs {
    CopySeg seg[kMaxCopySegs];
    uint32_t n;
};

// Queue one growing-stream staging kernel: copy every segment, copy
// meta_bytes (a multiple of 16, may be 0) from meta_src (pinned, coherent
// host memory) to meta_dst (device), and clear n_heads queue heads.
hipError_t launch_copy_stage(const CopySegs& segs, const void* meta_src, void* meta_dst,
                             uint32_t meta_bytes, uint32_t* heads, uint32_t n_heads,
                             hipStream_t stream);

// As launch_batch without the queue-head reset (the caller clears the head);
// part (device) receives the partial sums of sliced tiles (may be null when
// the launch has none).
hipError_t launch_batch_noreset(uint32_t bw, uint32_t threads, bool padded,
                                const BatchStream* streams, const BatchTile* tiles,
                                uint32_t n_tiles, uint32_t* head, uint32_t* part, uint32_t grid,
                                uint32_t lds_bytes, hipStream_t stream);

// Queue the combine step of n_jobs sliced pairs (after the batch launches
// that wrote their parts, on the same stream).  lds_bytes: (2qw + dn) * 4 of
// the largest shape among the jobs.  streams, jobs, part: device memory.
hipError_t launch_combine(const BatchStream* streams, const CombineJob* jobs, uint32_t n_jobs,
                          const uint32_t* part, uint32_t grid, uint32_t lds_bytes,
                          hipStream_t stream);

// As launch_combine for jobs of padded shapes, whose parts come from
// element slices (BatchTile with n_items elements from item0) and whose
// outputs may start at any byte; lds_bytes: (3qw + dn) * 4 of the largest
// shape among the jobs.
hipError_t launch_combine_padded(const BatchStream* streams, const CombineJob* jobs,
                                 uint32_t n_jobs, const uint32_t* part, uint32_t grid,
                                 uint32_t lds_bytes, hipStream_t stream);

// Queue the VALU issue-rate probe: blocks x kThreads lanes, each running
// iters * 16 * 9 VALU operations; out holds blocks * kThreads words.
hipError_t launch_valu_probe(uint32_t* out, uint32_t blocks, uint32_t iters, hipStream_t stream);
constexpr uint32_t kProbeOpsPerIter = 16 * 9;  // 8 AND-XORs and 1 funnel shift, 16 times

// Bit-sliced kernel for small fields (ext_bitslice.hip): 32 block pairs per
// 256-lane work-group, any q <= kBitsliceMaxQ divisible by 8, blocks and
// outputs at any byte offset.  bitslice_lds_words: its LDS need (the launch
// is refused above 64 KiB).
constexpr uint32_t kBitsliceMaxQ = 128;
uint32_t bitslice_lds_words(const ExtShape& s);
// Geometry of the bit-sliced kernel for s: elements per chunk, Karatsuba
// levels over the bit planes, planes per piece (q / 2^levels), and element
// subsets (lanes per sub-product).
void bitslice_describe(const ExtShape& s, uint32_t* chunk_elements, uint32_t* levels,
                       uint32_t* piece_planes, uint32_t* element_subsets);
hipError_t launch_bitslice(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                           uint64_t n_pairs, hipStream_t stream);

// Resident work-groups per CU of the batched kernel at this LDS size.
hipError_t batch_occupancy(uint32_t bw, uint32_t threads, bool padded, uint32_t lds_bytes,
                           int* blocks_per_cu);

// Static device scratch of the allocation-free growing-block call
// (ext_noalloc.hip): the launch tables of at most kNoAllocMaxBlocks blocks
// (one stream and one tile each) and kNoAllocMaxLaunches queue heads.
constexpr uint32_t kNoAllocMaxBlocks = 4096;
constexpr uint32_t kNoAllocMaxLaunches = 64;
constexpr size_t round256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kNoAllocStreamsOff = 0;
constexpr size_t kNoAllocTilesOff = round256(kNoAllocMaxBlocks * sizeof(BatchStream));
constexpr size_t kNoAllocHeadsOff =
    kNoAllocTilesOff + round256(kNoAllocMaxBlocks * sizeof(BatchTile));
constexpr size_t kNoAllocScratchBytes =
    kNoAllocHeadsOff + round256(kNoAllocMaxLaunches * sizeof(uint32_t));
// Look up this device's copy of the static scratch (once per device; the
// library calls it when a growing-block handle is created on the device).
hipError_t noalloc_scratch_init(int device);
// Device address of that copy, or null if it has not been looked up.
void* noalloc_scratch(int device);

}  // namespace qext
