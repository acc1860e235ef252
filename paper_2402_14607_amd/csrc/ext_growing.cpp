// ext_growing.cpp -- Algorithm 2 (Ext_bs^neq): blocks that grow by Delta
// samples' worth of field degree each.
//
// Block l (from 0) holds q_l * n_e bits of each source, right after block
// l-1, with q_l = q_1 + l * Delta * b, and yields Ext_IP^{n_e, q_l} of the
// two blocks (q_l output bits); the outputs are concatenated.  Every block
// has its own field, modulus and launch plan, so a call turns the first k
// blocks into k one-pair streams of the batched kernel (one persistent
// launch per base size) in the padded layout: block and output offsets are
// then byte-granular, whatever q_l is.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/qrng_ext.h"
#include "ext_internal.h"
#include "gf2_modulus.h"

using qext::BatchStream;
using qext::BatchTile;
using qext::ExtShape;

struct ext_growing {
    uint32_t n_e = 0, q1 = 0, delta_steps = 0, b = 8;
    ext_params params{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::map<uint32_t, ExtShape> shapes;  // plan per degree
    // device scratch, grown on demand
    BatchStream* d_streams = nullptr;
    BatchTile* d_tiles = nullptr;
    uint32_t* d_heads = nullptr;
    uint64_t cap_blocks = 0;
    uint8_t *dx = nullptr, *dy = nullptr, *dout = nullptr;  // host-memory mode
    uint64_t cap_in = 0, cap_out = 0;
    // the launches of one call (one per base size) are independent: they run
    // on lane streams forked from and joined back into `stream` with events
    static constexpr int kLanes = 4;
    hipStream_t lanes[kLanes] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t joins[kLanes] = {};
    int sticky = EXT_OK;
};

namespace {

constexpr uint32_t kMaxGroups = qext::kNoAllocMaxLaunches;  // distinct (base size, work-group
                                                            // size) launches per call

void release_lanes(ext_growing* g) {
    for (int i = 0; i < ext_growing::kLanes; ++i) {
        if (g->lanes[i]) {
            (void)hipStreamSynchronize(g->lanes[i]);
            (void)hipStreamDestroy(g->lanes[i]);
        }
        if (g->joins[i]) (void)hipEventDestroy(g->joins[i]);
        g->lanes[i] = nullptr;
        g->joins[i] = nullptr;
    }
    if (g->fork) (void)hipEventDestroy(g->fork);
    g->fork = nullptr;
}

void free_scratch(ext_growing* g) {
    (void)hipFree(g->d_streams);
    (void)hipFree(g->d_tiles);
    (void)hipFree(g->d_heads);
    (void)hipFree(g->dx);
    (void)hipFree(g->dy);
    (void)hipFree(g->dout);
    g->d_streams = nullptr;
    g->d_tiles = nullptr;
    g->d_heads = nullptr;
    g->dx = g->dy = g->dout = nullptr;
    g->cap_blocks = g->cap_in = g->cap_out = 0;
}

// Block geometry of the first k blocks: q_l, input offset and output offset.
struct Geo {
    uint64_t k = 0, in_bytes = 0, out_bytes = 0;
};

Geo geometry(const ext_growing* g, uint64_t n_bytes, uint64_t max_blocks) {
    Geo r;
    uint64_t q = g->q1;
    const uint64_t step = (uint64_t)g->delta_steps * g->b;
    while (r.k < max_blocks) {
        const uint64_t nb = q * g->n_e / 8;
        if (q > 0xffffffffull || r.in_bytes + nb > n_bytes) break;
        r.in_bytes += nb;
        r.out_bytes += q / 8;
        r.k += 1;
        q += step;
    }
    return r;
}

int plan_for(ext_growing* g, uint32_t q, ExtShape* out) {
    auto it = g->shapes.find(q);
    if (it != g->shapes.end()) {
        *out = it->second;
        return EXT_OK;
    }
    std::vector<uint32_t> taps;
    if (!qext::default_modulus(q, &taps)) return EXT_ENOTSUP;
    qext::PlanKnobs knobs{g->params.base_bits / 32, 0, 0, g->params.threads, 1};
    ExtShape s;
    if (!qext::plan_shape(q, g->n_e, taps.data(), (uint32_t)taps.size(), knobs, &s))
        return EXT_ENOTSUP;
    g->shapes[q] = s;
    *out = s;
    return EXT_OK;
}

int grow(ext_growing* g, uint64_t k, uint64_t in_bytes, uint64_t out_bytes) {
    bool ok = true;
    if (k > g->cap_blocks) {
        (void)hipFree(g->d_streams);
        (void)hipFree(g->d_tiles);
        g->d_streams = nullptr;
        g->d_tiles = nullptr;
        ok = hipMalloc((void**)&g->d_streams, k * sizeof(BatchStream)) == hipSuccess &&
             hipMalloc((void**)&g->d_tiles, k * sizeof(BatchTile)) == hipSuccess;
        g->cap_blocks = ok ? k : 0;
    }
    if (ok && !g->d_heads)
        ok = hipMalloc((void**)&g->d_heads, kMaxGroups * sizeof(uint32_t)) == hipSuccess;
    if (ok && g->params.mem_kind == EXT_MEM_HOST && in_bytes > g->cap_in) {
        (void)hipFree(g->dx);
        (void)hipFree(g->dy);
        g->dx = g->dy = nullptr;
        ok = hipMalloc((void**)&g->dx, in_bytes) == hipSuccess &&
             hipMalloc((void**)&g->dy, in_bytes) == hipSuccess;
        g->cap_in = ok ? in_bytes : 0;
    }
    if (ok && g->params.mem_kind == EXT_MEM_HOST && out_bytes > g->cap_out) {
        (void)hipFree(g->dout);
        g->dout = nullptr;
        ok = hipMalloc((void**)&g->dout, out_bytes) == hipSuccess;
        g->cap_out = ok ? out_bytes : 0;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_scratch(g);
        return EXT_ENOMEM;
    }
    return EXT_OK;
}

}  // namespace

extern "C" {

int ext_growing_create(uint32_t n_e, uint32_t q1, uint32_t delta_steps, const ext_params* p,
                       ext_growing** out) {
    if (!out) return EXT_EINVAL;
    *out = nullptr;
    ext_params def;
    ext_params_init(&def);
    if (!p) p = &def;
    const uint32_t b = p->sample_bits ? p->sample_bits : 8;
    if (n_e == 0 || q1 == 0 || q1 % 8 || q1 % b || ((uint64_t)delta_steps * b) % 8 || p->n_taps)
        return EXT_EINVAL;
    if (p->mem_kind != EXT_MEM_HOST && p->mem_kind != EXT_MEM_DEVICE) return EXT_EINVAL;
    if (p->kernel > EXT_KERNEL_BITSLICE) return EXT_EINVAL;
    if (p->kernel == EXT_KERNEL_BITSLICE) return EXT_ENOTSUP;  // word-level kernels only
    if (p->base_bits % 32) return EXT_EINVAL;
    ext_growing* g = new (std::nothrow) ext_growing;
    if (!g) return EXT_ENOMEM;
    g->n_e = n_e;
    g->q1 = q1;
    g->delta_steps = delta_steps;
    g->b = b;
    g->params = *p;
    int dev = p->device;
    if ((dev < 0 && hipGetDevice(&dev) != hipSuccess) || hipSetDevice(dev) != hipSuccess) {
        delete g;
        return EXT_EDEVICE;
    }
    g->device = dev;
    // set-up of the allocation-free call: this device's copy of the static
    // scratch (a failure leaves only that call unusable)
    (void)qext::noalloc_scratch_init(dev);
    if (p->use_hip_stream) {
        g->stream = (hipStream_t)p->hip_stream;
    } else if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) == hipSuccess) {
        g->own_stream = true;
    } else {
        delete g;
        return EXT_EDEVICE;
    }
    bool ok = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < ext_growing::kLanes; ++i)
        ok = hipStreamCreateWithFlags(&g->lanes[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&g->joins[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        release_lanes(g);
        if (g->own_stream) (void)hipStreamDestroy(g->stream);
        delete g;
        return EXT_EDEVICE;
    }
    *out = g;
    return EXT_OK;
}

int ext_growing_blocks(const ext_growing* g, uint64_t n_bytes, uint64_t* k_blocks,
                       uint64_t* in_bytes, uint64_t* out_bytes) {
    if (!g) return EXT_EINVAL;
    const Geo r = geometry(g, n_bytes, ~0ull);
    if (k_blocks) *k_blocks = r.k;
    if (in_bytes) *in_bytes = r.in_bytes;
    if (out_bytes) *out_bytes = r.out_bytes;
    return EXT_OK;
}

}  // extern "C"

namespace {

// Where a call's launch tables and queue heads live on the device.
struct Tables {
    BatchStream* streams;
    BatchTile* tiles;
    uint32_t* heads;
};

// Blocks 0 .. k-1 of x and y into out (ext_growing_extract); the launch
// tables go to *fixed when given (nothing is allocated then), else to the
// handle's scratch, grown on demand.
int extract_blocks(ext_growing* g, const void* x, const void* y, uint64_t n_bytes,
                   uint64_t max_blocks, void* out, uint64_t out_cap, uint64_t* n_blocks,
                   const Tables* fixed) {
    if (!g) return EXT_EINVAL;
    if (g->sticky) return g->sticky;
    if (n_blocks) *n_blocks = 0;
    const Geo r = geometry(g, n_bytes, max_blocks);
    if (r.k == 0) return EXT_OK;
    if (!x || !y || !out || out_cap < r.out_bytes) return EXT_EINVAL;
    if (fixed && r.k > qext::kNoAllocMaxBlocks) return EXT_ENOMEM;
    if (hipSetDevice(g->device) != hipSuccess) return EXT_EDEVICE;
    int rc = EXT_OK;
    std::vector<BatchStream> streams;
    std::vector<BatchTile> tiles;
    // launches: (base size, work-group size) -> tile list with cost
    std::map<std::pair<uint32_t, uint32_t>, std::vector<std::pair<uint64_t, uint32_t>>> groups;
    try {
        streams.reserve(r.k);
        Tables tab;
        if (fixed) {
            tab = *fixed;
        } else {
            rc = grow(g, r.k, r.in_bytes, r.out_bytes);
            if (rc) return rc;
            tab = Tables{g->d_streams, g->d_tiles, g->d_heads};
        }
        const bool host = g->params.mem_kind == EXT_MEM_HOST;
        const uint8_t* xs = host ? g->dx : (const uint8_t*)x;
        const uint8_t* ys = host ? g->dy : (const uint8_t*)y;
        uint8_t* os = host ? g->dout : (uint8_t*)out;
        uint64_t q = g->q1, in_off = 0, out_off = 0;
        for (uint64_t l = 0; l < r.k; ++l) {
            ExtShape s;
            rc = plan_for(g, (uint32_t)q, &s);
            if (rc) return rc;
            streams.push_back(BatchStream{xs + in_off, ys + in_off, os + out_off, 1, s});
            const uint64_t cost = ((uint64_t)s.np * s.groups + s.threads - 1) / s.threads * s.epg;
            groups[{s.bw, s.threads}].push_back({cost, (uint32_t)l});
            in_off += s.nbytes;
            out_off += s.qbytes;
            q += (uint64_t)g->delta_steps * g->b;
        }
        if (groups.size() > kMaxGroups) return EXT_ENOTSUP;
        // from here on work is queued: every exit waits for the stream first,
        // so no copy still reads the caller's or these host buffers
        auto device_error = [&]() {
            for (int i = 0; i < ext_growing::kLanes; ++i) (void)hipStreamSynchronize(g->lanes[i]);
            (void)hipStreamSynchronize(g->stream);
            (void)hipGetLastError();
            return g->sticky = EXT_EDEVICE;
        };
        if (host) {
            if (hipMemcpyAsync(g->dx, x, r.in_bytes, hipMemcpyHostToDevice, g->stream) ||
                hipMemcpyAsync(g->dy, y, r.in_bytes, hipMemcpyHostToDevice, g->stream))
                return device_error();
        }
        int cus = 1;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device);
        struct L {
            uint32_t bw, threads, off, n, lds, grid;
            uint64_t cost;  // sum of its tiles' costs
        };
        std::vector<L> launches;
        for (auto& kv : groups) {
            auto& v = kv.second;
            // longest tiles first, so the queue ends with short ones
            std::stable_sort(v.begin(), v.end(),
                             [](const auto& a, const auto& c) { return a.first > c.first; });
            L ln{kv.first.first, kv.first.second, (uint32_t)tiles.size(), (uint32_t)v.size(), 0, 0, 0};
            for (auto& t : v) {
                ln.cost += t.first;
                tiles.push_back(BatchTile{t.second, 1, 0, 0, 0, 0});
                ln.lds = std::max(ln.lds, streams[t.second].shape.lds_words * 4);
            }
            int occ = 0;
            if (qext::batch_occupancy(ln.bw, ln.threads, true, ln.lds, &occ) != hipSuccess || occ <= 0)
                occ = 1;
            ln.grid = (uint32_t)std::min<uint64_t>(ln.n, (uint64_t)cus * occ);
            launches.push_back(ln);
        }
        // the tables and the launches' zeroed queue heads, in stream order
        // before the lanes fork (a copy, so that no launch needs a reset kernel)
        static const uint32_t kZeroHeads[kMaxGroups] = {};
        if (hipMemcpyAsync(tab.streams, streams.data(), r.k * sizeof(BatchStream),
                           hipMemcpyHostToDevice, g->stream) ||
            hipMemcpyAsync(tab.tiles, tiles.data(), r.k * sizeof(BatchTile),
                           hipMemcpyHostToDevice, g->stream) ||
            hipMemcpyAsync(tab.heads, kZeroHeads, launches.size() * sizeof(uint32_t),
                           hipMemcpyHostToDevice, g->stream))
            return device_error();
        // fork: the lanes start after the table copies (and the caller's work
        // queued before this call); costliest launches first, each on the
        // least loaded lane; join: the stream waits for every lane used
        if (hipEventRecord(g->fork, g->stream) != hipSuccess) return device_error();
        std::vector<size_t> order(launches.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t c) { return launches[a].cost > launches[c].cost; });
        uint64_t load[ext_growing::kLanes] = {};
        bool used[ext_growing::kLanes] = {};
        for (size_t i : order) {
            const L& ln = launches[i];
            int lane = 0;
            for (int l = 1; l < ext_growing::kLanes; ++l)
                if (load[l] < load[lane]) lane = l;
            if (!used[lane] && hipStreamWaitEvent(g->lanes[lane], g->fork, 0) != hipSuccess)
                return device_error();
            used[lane] = true;
            load[lane] += ln.cost + 1;
            if (qext::launch_batch_noreset(ln.bw, ln.threads, true, tab.streams,
                                           tab.tiles + ln.off, ln.n, tab.heads + i, nullptr,
                                           ln.grid, ln.lds, g->lanes[lane]) != hipSuccess)
                return device_error();
        }
        for (int l = 0; l < ext_growing::kLanes; ++l) {
            if (!used[l]) continue;
            if (hipEventRecord(g->joins[l], g->lanes[l]) != hipSuccess ||
                hipStreamWaitEvent(g->stream, g->joins[l], 0) != hipSuccess)
                return device_error();
        }
        if (host && hipMemcpyAsync(out, g->dout, r.out_bytes, hipMemcpyDeviceToHost, g->stream))
            return device_error();
        // the host vectors above are read by the copies: wait before they go
        if (hipStreamSynchronize(g->stream) != hipSuccess) return g->sticky = EXT_EDEVICE;
    } catch (const std::bad_alloc&) {
        return EXT_ENOMEM;
    }
    if (n_blocks) *n_blocks = r.k;
    return EXT_OK;
}

}  // namespace

extern "C" {

int ext_growing_extract(ext_growing* g, const void* x, const void* y, uint64_t n_bytes,
                        uint64_t max_blocks, void* out, uint64_t out_cap, uint64_t* n_blocks) {
    return extract_blocks(g, x, y, n_bytes, max_blocks, out, out_cap, n_blocks, nullptr);
}

int ext_growing_extract_noalloc(ext_growing* g, const void* x, const void* y, uint64_t n_bytes,
                                uint64_t max_blocks, void* out, uint64_t out_cap,
                                uint64_t* n_blocks) {
    if (!g) return EXT_EINVAL;
    // host memory would need device staging buffers
    if (g->params.mem_kind != EXT_MEM_DEVICE) return EXT_EINVAL;
    uint8_t* base = (uint8_t*)qext::noalloc_scratch(g->device);
    if (!base) return EXT_EDEVICE;  // the per-device lookup at create time failed
    const Tables tab{(BatchStream*)(base + qext::kNoAllocStreamsOff),
                     (BatchTile*)(base + qext::kNoAllocTilesOff),
                     (uint32_t*)(base + qext::kNoAllocHeadsOff)};
    return extract_blocks(g, x, y, n_bytes, max_blocks, out, out_cap, n_blocks, &tab);
}

int ext_growing_destroy(ext_growing* g) {
    if (!g) return EXT_EINVAL;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release_lanes(g);
    free_scratch(g);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return EXT_OK;
}

}  // extern "C"
