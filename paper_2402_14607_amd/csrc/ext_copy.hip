// ext_copy.hip -- the staging kernel of the online growing-block form: one
// launch that moves a submission's bytes into the pending buffers, uploads a
// call's launch tables from pinned host memory and clears its queue heads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ext_internal.h"

namespace qext {
namespace {

constexpr uint32_t kCopyThreads = 256;

// Copy len bytes from src to dst with the grid's lanes (gid of gsz): 16-byte
// accesses when the two addresses agree modulo 16, 4-byte ones when they
// agree modulo 4, else bytes; the unaligned head and tail go byte by byte.
__device__ __forceinline__ void copy_range(const uint8_t* __restrict__ src,
                                           uint8_t* __restrict__ dst, uint64_t len, uint64_t gid,
                                           uint64_t gsz) {
    const uintptr_t mis = ((uintptr_t)src ^ (uintptr_t)dst);
    const uint32_t unit = (mis & 15u) == 0 ? 16u : ((mis & 3u) == 0 ? 4u : 1u);
    uint64_t head = (unit - ((uintptr_t)dst & (unit - 1u))) & (unit - 1u);
    head = head < len ? head : len;
    const uint64_t body = (len - head) / unit;
    const uint64_t tail0 = head + body * unit;
    for (uint64_t i = gid; i < head; i += gsz) dst[i] = src[i];
    for (uint64_t i = tail0 + gid; i < len; i += gsz) dst[i] = src[i];
    if (unit == 16u) {
        const uint4* s16 = reinterpret_cast<const uint4*>(src + head);
        uint4* t16 = reinterpret_cast<uint4*>(dst + head);
        uint64_t i = gid;
        for (; i + 3 * gsz < body; i += 4 * gsz) {  // four loads in flight per lane
            const uint4 a = s16[i];
            const uint4 b = s16[i + gsz];
            const uint4 c = s16[i + 2 * gsz];
            const uint4 d = s16[i + 3 * gsz];
            t16[i] = a;
            t16[i + gsz] = b;
            t16[i + 2 * gsz] = c;
            t16[i + 3 * gsz] = d;
        }
        for (; i < body; i += gsz) t16[i] = s16[i];
    } else if (unit == 4u) {
        const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src + head);
        uint32_t* t4 = reinterpret_cast<uint32_t*>(dst + head);
        for (uint64_t i = gid; i < body; i += gsz) t4[i] = s4[i];
    } else {
        for (uint64_t i = gid; i < body; i += gsz) dst[head + i] = src[head + i];
    }
}

// Start of a growing-stream call: the grid copies the byte segments (pending
// input compaction and newly submitted chunks), copies the call's launch
// tables from pinned host memory, and work-group 0 clears the queue heads --
// one kernel where separate copies would each cost a runtime call.
__global__ void __launch_bounds__(kCopyThreads)
copy_stage_kernel(CopySegs segs, const uint4* __restrict__ meta_src, uint4* __restrict__ meta_dst,
                  uint32_t meta_vec, uint32_t* __restrict__ heads, uint32_t n_heads) {
    const uint64_t gid = (uint64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    const uint64_t gsz = (uint64_t)gridDim.x * kCopyThreads;
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < n_heads; i += kCopyThreads) heads[i] = 0u;
    for (uint64_t i = gid; i < meta_vec; i += gsz) meta_dst[i] = meta_src[i];
    for (uint32_t k = 0; k < segs.n; ++k)
        copy_range(segs.seg[k].src, segs.seg[k].dst, segs.seg[k].len, gid, gsz);
}

}  // namespace

hipError_t launch_copy_stage(const CopySegs& segs, const void* meta_src, void* meta_dst,
                             uint32_t meta_bytes, uint32_t* heads, uint32_t n_heads,
                             hipStream_t stream) {
    if (meta_bytes % 16 || segs.n > kMaxCopySegs || (meta_bytes && (!meta_src || !meta_dst)) ||
        (n_heads && !heads))
        return hipErrorInvalidValue;
    uint64_t bytes = meta_bytes;
    for (uint32_t k = 0; k < segs.n; ++k) {
        if (segs.seg[k].len && (!segs.seg[k].src || !segs.seg[k].dst)) return hipErrorInvalidValue;
        bytes += segs.seg[k].len;
    }
    if (bytes == 0 && n_heads == 0) return hipSuccess;
    // about 4 KiB per work-group: one 16-byte move per lane and segment, so
    // that the copy takes about one round trip per segment
    uint64_t grid = (bytes + 4095) / 4096;
    grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
    hipLaunchKernelGGL(copy_stage_kernel, dim3((uint32_t)grid), dim3(kCopyThreads), 0, stream, segs,
                       static_cast<const uint4*>(meta_src), static_cast<uint4*>(meta_dst),
                       meta_bytes / 16, heads, n_heads);
    return hipGetLastError();
}

}  // namespace qext
