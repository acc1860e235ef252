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
//
// The online form (ext_growing_open / submit / poll / close) runs Algorithm 2
// on unbounded sources: its state (the next block l, its degree q_l and the
// bytes consumed so far, i of Algorithm 2) carries over from call to call,
// the bytes of the block still incomplete wait in device buffers, and every
// submission launches the blocks it completes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/qrng_ext.h"
#include "ext_internal.h"
#include "gf2_modulus.h"

using qext::BatchStream;
using qext::BatchTile;
using qext::CombineJob;
using qext::ExtShape;

namespace {

// Launch plan of one degree: the whole-block shape when one work-group can
// hold a block, and the slice geometry (elements per slice) used for blocks
// too large for that, or large enough that slicing fills more of the GPU.
struct DegreePlan {
    ExtShape whole{};
    bool whole_ok = false;
    ExtShape sliced{};  // the padded element geometry of the degree, n_e of the block
    uint32_t slice_elems = 0;  // 0: the degree cannot be sliced
};

}  // namespace

struct ext_growing {
    uint32_t n_e = 0, q1 = 0, delta_steps = 0, b = 8;
    ext_params params{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::map<uint32_t, DegreePlan> plans;  // plan per degree
    // launch tables of the prefix call, packed (streams, tiles, jobs), in
    // device memory and in pinned, coherent host memory that the staging
    // kernel reads; grown on demand
    uint8_t* d_tab = nullptr;
    uint8_t* h_tab = nullptr;
    uint64_t cap_tab = 0;
    uint32_t* d_heads = nullptr;
    // partial sums of sliced blocks (every call of the handle, in stream order)
    uint32_t* d_part = nullptr;
    uint64_t cap_part = 0;
    uint8_t *dx = nullptr, *dy = nullptr, *dout = nullptr;  // host-memory mode
    uint64_t cap_in = 0, cap_out = 0;
    // the launches of one call (one per base size) are independent: they run
    // on lane streams forked from and joined back into `stream` with events
    static constexpr int kLanes = 4;
    hipStream_t lanes[kLanes] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t joins[kLanes] = {};
    hipStream_t copy = nullptr;  // online form: outputs back to the caller
    std::vector<ext_growing_stream*> open_streams;
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
    if (g->copy) (void)hipStreamDestroy(g->copy);
    g->copy = nullptr;
}

void free_scratch(ext_growing* g) {
    (void)hipFree(g->d_tab);
    if (g->h_tab) (void)hipHostFree(g->h_tab);
    (void)hipFree(g->d_heads);
    (void)hipFree(g->d_part);
    (void)hipFree(g->dx);
    (void)hipFree(g->dy);
    (void)hipFree(g->dout);
    g->d_tab = nullptr;
    g->h_tab = nullptr;
    g->d_heads = nullptr;
    g->d_part = nullptr;
    g->dx = g->dy = g->dout = nullptr;
    g->cap_tab = g->cap_part = 0;
    g->cap_in = g->cap_out = 0;
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

// Most LDS words a slice may take (its two staged element ranges and the
// partial sum), and slot words per lane of the padded staging.
constexpr uint32_t kSliceLdsWords = 12288;

int plan_for(ext_growing* g, uint32_t q, DegreePlan* out) {
    auto it = g->plans.find(q);
    if (it != g->plans.end()) {
        *out = it->second;
        return EXT_OK;
    }
    std::vector<uint32_t> taps;
    if (!qext::default_modulus(q, &taps)) return EXT_ENOTSUP;
    // odd parts up to 7: base products of at most 8 words.  A block is one
    // pair, so a call is bound by the longest lane's chain of AND-XORs; over
    // q = 80 .. 5184 this padding rule also does slightly less work in total
    // than odd parts up to 15 (deeper Karatsuba makes up for the padding).
    qext::PlanKnobs knobs{g->params.base_bits / 32, 0, 0, g->params.threads, 1, 7};
    DegreePlan d;
    d.whole_ok = qext::plan_shape(q, g->n_e, taps.data(), (uint32_t)taps.size(), knobs, &d.whole);
    // slices: the degree's geometry for one element, then the block's n_e
    ExtShape u;
    if (qext::plan_shape(q, 1, taps.data(), (uint32_t)taps.size(), knobs, &u)) {
        u.n_e = g->n_e;
        u.nw = u.qw * g->n_e;
        u.nbytes = (uint32_t)((uint64_t)g->n_e * q / 8);
        // one round of items per slice, within the LDS and staging budgets
        uint32_t es = std::max<uint32_t>(1u, u.threads / u.np);
        const uint32_t by_lds =
            (2 * u.qw + 2 * qext::kPadSlack) < kSliceLdsWords
                ? (kSliceLdsWords - 2 * u.qw - 2 * qext::kPadSlack) / (2 * u.qw)
                : 0u;
        const uint32_t by_regs = qext::kPadRegs * u.threads / u.qw;
        es = std::min({es, by_lds, by_regs, g->n_e});
        if (es > 0) {
            const uint32_t parts = (g->n_e + es - 1) / es;
            d.slice_elems = (g->n_e + parts - 1) / parts;  // even slices
            d.sliced = u;
        }
    }
    if (!d.whole_ok && !d.slice_elems) return EXT_ENOTSUP;
    g->plans[q] = d;
    *out = d;
    return EXT_OK;
}

// Whether a block of degree plan d is computed in slices: when no single
// work-group can hold it, or when its items fill more than two rounds of a
// work-group's lanes (slices then spread it over the GPU).
bool use_slices(const DegreePlan& d, bool allow) {
    if (!d.whole_ok) return true;
    if (!allow || !d.slice_elems) return false;
    return (uint64_t)d.whole.np * d.whole.n_e > 2ull * d.whole.threads;
}

// Table buffers of the prefix call, grown to at least `bytes` each (every
// prefix call waits for its work before returning, so none is in use).
int grow_tables(ext_growing* g, uint64_t bytes) {
    bool ok = true;
    if (bytes > g->cap_tab) {
        (void)hipFree(g->d_tab);
        if (g->h_tab) (void)hipHostFree(g->h_tab);
        g->d_tab = nullptr;
        g->h_tab = nullptr;
        g->cap_tab = 0;
        ok = hipMalloc((void**)&g->d_tab, bytes) == hipSuccess &&
             hipHostMalloc((void**)&g->h_tab, bytes, hipHostMallocCoherent) == hipSuccess;
        if (ok) g->cap_tab = bytes;
    }
    if (ok && !g->d_heads)
        ok = hipMalloc((void**)&g->d_heads, kMaxGroups * sizeof(uint32_t)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return EXT_ENOMEM;
    }
    return EXT_OK;
}

// The handle's partial-sum buffer, grown to at least `words` (after the
// queued work that may use the old one).
int grow_part(ext_growing* g, uint64_t words) {
    if (words <= g->cap_part) return EXT_OK;
    if (hipStreamSynchronize(g->stream) != hipSuccess) {
        (void)hipGetLastError();
        return g->sticky = EXT_EDEVICE;
    }
    const uint64_t want = std::max<uint64_t>(words, 2 * g->cap_part);
    (void)hipFree(g->d_part);
    g->d_part = nullptr;
    g->cap_part = 0;
    if (hipMalloc((void**)&g->d_part, want * 4) != hipSuccess) {
        (void)hipGetLastError();
        return EXT_ENOMEM;
    }
    g->cap_part = want;
    return EXT_OK;
}

// Input and output staging of the prefix call in host-memory mode.
int grow_io(ext_growing* g, uint64_t in_bytes, uint64_t out_bytes) {
    bool ok = true;
    if (g->params.mem_kind == EXT_MEM_HOST && in_bytes > g->cap_in) {
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
    bool ok = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&g->copy, hipStreamNonBlocking) == hipSuccess;
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
    CombineJob* jobs;
    uint32_t* heads;
};

constexpr size_t round16(size_t v) { return (v + 15) / 16 * 16; }

// One persistent launch of a planned call: the tiles [off, off + n) of one
// (base size, work-group size) class.
struct LaunchPlan {
    uint32_t bw, threads, off, n, lds, grid;
    uint64_t cost;  // sum of its tiles' costs
};

// A planned call: one one-pair stream per block, one tile per whole block or
// one per slice of a sliced block, grouped into launches; one combine job per
// sliced block, whose parts take part_words words.
struct Planned {
    std::vector<BatchStream> streams;
    std::vector<BatchTile> tiles;
    std::vector<LaunchPlan> launches;
    std::vector<CombineJob> jobs;
    uint64_t part_words = 0;
    uint32_t combine_lds = 0;
};

// Plan k consecutive blocks of degrees q0, q0 + step, ... whose inputs start
// at xs / ys and whose outputs start at os (device addresses); allow_slices
// false plans whole blocks only (EXT_ENOTSUP for a block one work-group
// cannot hold).  May throw std::bad_alloc.
int plan_blocks(ext_growing* g, uint64_t q0, uint64_t k, const uint8_t* xs, const uint8_t* ys,
                uint8_t* os, bool allow_slices, Planned* p) {
    p->streams.clear();
    p->tiles.clear();
    p->launches.clear();
    p->jobs.clear();
    p->part_words = 0;
    p->combine_lds = 0;
    p->streams.reserve(k);
    // launches: (base size, work-group size) -> tiles with cost
    struct Group {
        std::vector<std::pair<uint64_t, BatchTile>> tiles;
        uint32_t lds = 0;
    };
    std::map<std::pair<uint32_t, uint32_t>, Group> groups;
    uint64_t q = q0, in_off = 0, out_off = 0;
    for (uint64_t l = 0; l < k; ++l) {
        if (q > 0xffffffffull) return EXT_ENOTSUP;
        DegreePlan d;
        const int rc = plan_for(g, (uint32_t)q, &d);
        if (rc) return rc;
        const bool sliced = use_slices(d, allow_slices);
        if (sliced && (!allow_slices || !d.slice_elems)) return EXT_ENOTSUP;
        const ExtShape& s = sliced ? d.sliced : d.whole;
        p->streams.push_back(BatchStream{xs + in_off, ys + in_off, os + out_off, 1, s});
        Group& gr = groups[{s.bw, s.threads}];
        if (!sliced) {
            const uint64_t cost = ((uint64_t)s.np * s.groups + s.threads - 1) / s.threads * s.epg;
            gr.tiles.push_back({cost, BatchTile{(uint32_t)l, 1, 0, 0, 0, 0}});
            gr.lds = std::max(gr.lds, qext::group_lds_bytes(s));
        } else {
            const uint32_t es = d.slice_elems, cw = 2 * s.qw;
            const uint32_t n_parts = (s.n_e + es - 1) / es;
            for (uint32_t e0 = 0, part = 0; e0 < s.n_e; e0 += es, ++part) {
                const uint32_t ne = std::min(es, s.n_e - e0);
                const uint64_t cost = ((uint64_t)s.np * ne + s.threads - 1) / s.threads;
                gr.tiles.push_back({cost, BatchTile{(uint32_t)l, 1, 0, p->part_words + part * cw,
                                                    e0, ne}});
            }
            gr.lds = std::max(gr.lds, (2 * (es * s.qw + qext::kPadSlack) + cw) * 4);
            p->jobs.push_back(CombineJob{(uint32_t)l, n_parts, p->part_words, 0});
            p->part_words += (uint64_t)n_parts * cw;
            p->combine_lds = std::max(p->combine_lds, (3 * s.qw + s.dn) * 4);
        }
        in_off += s.nbytes;
        out_off += s.qbytes;
        q += (uint64_t)g->delta_steps * g->b;
    }
    if (groups.size() > kMaxGroups) return EXT_ENOTSUP;
    if (p->combine_lds > 65536) return EXT_ENOTSUP;
    int cus = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device);
    for (auto& kv : groups) {
        auto& v = kv.second.tiles;
        // longest tiles first, so the queue ends with short ones
        std::stable_sort(v.begin(), v.end(),
                         [](const auto& a, const auto& c) { return a.first > c.first; });
        LaunchPlan ln{kv.first.first, kv.first.second, (uint32_t)p->tiles.size(),
                      (uint32_t)v.size(), kv.second.lds, 0, 0};
        for (auto& t : v) {
            ln.cost += t.first;
            p->tiles.push_back(t.second);
        }
        if (ln.lds > 65536) return EXT_ENOTSUP;
        int occ = 0;
        if (qext::batch_occupancy(ln.bw, ln.threads, true, ln.lds, &occ) != hipSuccess || occ <= 0)
            occ = 1;
        ln.grid = (uint32_t)std::min<uint64_t>(ln.n, (uint64_t)cus * occ);
        p->launches.push_back(ln);
    }
    return EXT_OK;
}

// Queue a planned call's launches on g->stream, its tables and zeroed queue
// heads already queued into tab: the costliest launch on g->stream itself,
// the others (one per further base size) on lanes forked from it at this
// point, each on the least loaded one, joined back before the combine step
// of the sliced blocks (their parts in g->d_part), which runs on g->stream.
// A call with one launch needs no fork or join.  On a HIP error the work
// queued so far is waited for and the handle's sticky error set.
int device_error(ext_growing* g) {
    for (int i = 0; i < ext_growing::kLanes; ++i) (void)hipStreamSynchronize(g->lanes[i]);
    (void)hipStreamSynchronize(g->stream);
    (void)hipGetLastError();
    return g->sticky = EXT_EDEVICE;
}

int queue_launches(ext_growing* g, const Planned& p, const Tables& tab) {
    std::vector<size_t> order(p.launches.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) {
        return p.launches[a].cost > p.launches[c].cost;
    });
    if (order.size() > 1 && hipEventRecord(g->fork, g->stream) != hipSuccess)
        return device_error(g);
    // lane 0 is g->stream, lane l > 0 is g->lanes[l - 1]
    uint64_t load[ext_growing::kLanes + 1] = {};
    bool used[ext_growing::kLanes + 1] = {};
    for (size_t i : order) {
        const LaunchPlan& ln = p.launches[i];
        int lane = 0;
        for (int l = 1; l <= ext_growing::kLanes; ++l)
            if (load[l] < load[lane]) lane = l;
        hipStream_t st = lane ? g->lanes[lane - 1] : g->stream;
        if (lane && !used[lane] && hipStreamWaitEvent(st, g->fork, 0) != hipSuccess)
            return device_error(g);
        used[lane] = true;
        load[lane] += ln.cost + 1;
        if (qext::launch_batch_noreset(ln.bw, ln.threads, true, tab.streams, tab.tiles + ln.off,
                                       ln.n, tab.heads + i, g->d_part, ln.grid, ln.lds,
                                       st) != hipSuccess)
            return device_error(g);
    }
    for (int l = 1; l <= ext_growing::kLanes; ++l) {
        if (!used[l]) continue;
        if (hipEventRecord(g->joins[l - 1], g->lanes[l - 1]) != hipSuccess ||
            hipStreamWaitEvent(g->stream, g->joins[l - 1], 0) != hipSuccess)
            return device_error(g);
    }
    if (!p.jobs.empty()) {
        int cus = 1;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device);
        const uint32_t grid = (uint32_t)std::min<uint64_t>(p.jobs.size(), (uint64_t)cus * 4);
        if (qext::launch_combine_padded(tab.streams, tab.jobs, (uint32_t)p.jobs.size(), g->d_part,
                                        grid, p.combine_lds, g->stream) != hipSuccess)
            return device_error(g);
    }
    return EXT_OK;
}

// Queue a planned call on g->stream: copies of its tables (read from host
// memory at streams_src, tiles_src and jobs_src, which must stay untouched
// until the copies have run) and of zeroed queue heads into tab, then its
// launches (queue_launches).
int queue_blocks(ext_growing* g, const Planned& p, const Tables& tab, const void* streams_src,
                 const void* tiles_src, const void* jobs_src) {
    // the queue heads are zeroed by a copy, so that no launch needs a reset kernel
    static const uint32_t kZeroHeads[kMaxGroups] = {};
    if (hipMemcpyAsync(tab.streams, streams_src, p.streams.size() * sizeof(BatchStream),
                       hipMemcpyHostToDevice, g->stream) ||
        hipMemcpyAsync(tab.tiles, tiles_src, p.tiles.size() * sizeof(BatchTile),
                       hipMemcpyHostToDevice, g->stream) ||
        (!p.jobs.empty() &&
         hipMemcpyAsync(tab.jobs, jobs_src, p.jobs.size() * sizeof(CombineJob),
                        hipMemcpyHostToDevice, g->stream)) ||
        hipMemcpyAsync(tab.heads, kZeroHeads, p.launches.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice, g->stream))
        return device_error(g);
    return queue_launches(g, p, tab);
}

// Blocks 0 .. k-1 of x and y into out (ext_growing_extract); the launch
// tables go to *fixed when given (nothing is allocated then, and every block
// must fit one work-group), else to the handle's scratch, grown on demand.
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
    try {
        const bool host = g->params.mem_kind == EXT_MEM_HOST;
        if (!fixed) {
            const int rc = grow_io(g, r.in_bytes, r.out_bytes);
            if (rc) return rc;
        }
        const uint8_t* xs = host ? g->dx : (const uint8_t*)x;
        const uint8_t* ys = host ? g->dy : (const uint8_t*)y;
        uint8_t* os = host ? g->dout : (uint8_t*)out;
        Planned p;
        int rc = plan_blocks(g, g->q1, r.k, xs, ys, os, !fixed, &p);
        if (rc) return rc;
        // the tables: copied into the static scratch (allocation-free call), or
        // packed into the handle's pinned buffer for the staging kernel
        Tables tab;
        size_t tab_bytes = 0;
        if (fixed) {
            tab = *fixed;
        } else {
            const size_t sb = p.streams.size() * sizeof(BatchStream);
            const size_t tb = p.tiles.size() * sizeof(BatchTile);
            const size_t jb = p.jobs.size() * sizeof(CombineJob);
            const size_t to = round16(sb), jo = to + round16(tb);
            tab_bytes = jo + round16(jb);
            if (tab_bytes > 0xffffffffull) return EXT_ENOTSUP;
            rc = grow_tables(g, tab_bytes);
            if (rc) return rc;
            rc = grow_part(g, p.part_words);
            if (rc) return rc;
            memcpy(g->h_tab, p.streams.data(), sb);
            memcpy(g->h_tab + to, p.tiles.data(), tb);
            memcpy(g->h_tab + jo, p.jobs.data(), jb);
            tab = Tables{(BatchStream*)g->d_tab, (BatchTile*)(g->d_tab + to),
                         (CombineJob*)(g->d_tab + jo), g->d_heads};
        }
        // from here on work is queued: every exit waits for the stream first,
        // so no copy still reads the caller's or these host buffers
        if (host) {
            if (hipMemcpyAsync(g->dx, x, r.in_bytes, hipMemcpyHostToDevice, g->stream) ||
                hipMemcpyAsync(g->dy, y, r.in_bytes, hipMemcpyHostToDevice, g->stream)) {
                (void)hipStreamSynchronize(g->stream);
                (void)hipGetLastError();
                return g->sticky = EXT_EDEVICE;
            }
        }
        if (fixed) {
            rc = queue_blocks(g, p, tab, p.streams.data(), p.tiles.data(), p.jobs.data());
        } else {
            // one staging kernel uploads the tables and clears the queue heads
            if (qext::launch_copy_stage(qext::CopySegs{}, g->h_tab, g->d_tab, (uint32_t)tab_bytes,
                                        g->d_heads, (uint32_t)p.launches.size(),
                                        g->stream) != hipSuccess)
                return device_error(g);
            rc = queue_launches(g, p, tab);
        }
        if (rc) return rc;
        if (host && hipMemcpyAsync(out, g->dout, r.out_bytes, hipMemcpyDeviceToHost, g->stream)) {
            (void)hipStreamSynchronize(g->stream);
            (void)hipGetLastError();
            return g->sticky = EXT_EDEVICE;
        }
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
                     (BatchTile*)(base + qext::kNoAllocTilesOff), nullptr,
                     (uint32_t*)(base + qext::kNoAllocHeadsOff)};
    return extract_blocks(g, x, y, n_bytes, max_blocks, out, out_cap, n_blocks, &tab);
}

int ext_growing_destroy(ext_growing* g) {
    if (!g) return EXT_EINVAL;
    (void)hipSetDevice(g->device);
    while (!g->open_streams.empty()) (void)ext_growing_close(g->open_streams.back(), nullptr);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release_lanes(g);
    free_scratch(g);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
    return EXT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// online form
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kMaxLaunchBlocks = 1024;  // blocks per queued call
constexpr uint64_t kMaxLaunchTiles = 16384;  // tiles per queued call (slices count each)
// the largest table set of one call, packed: streams, tiles, jobs
constexpr size_t kTableBytes = round16(kMaxLaunchBlocks * sizeof(BatchStream)) +
                               round16(kMaxLaunchTiles * sizeof(BatchTile)) +
                               round16(kMaxLaunchBlocks * sizeof(CombineJob));

// One queued call of the online form: k blocks from block0 (degree q0), their
// outputs at monotonic ring position opos.
struct GLaunch {
    uint64_t block0, k, q0;
    uint64_t opos, obytes;
    uint64_t taken = 0, taken_bytes = 0;  // blocks and bytes returned by poll
    hipEvent_t done = nullptr;
};

}  // namespace

struct ext_growing_stream {
    ext_growing* g = nullptr;
    uint64_t step = 0;  // Delta * b, bits of degree added per block
    // Algorithm 2's state: the next block l, its degree q_l, and i (bytes per
    // source of blocks 0 .. l-1)
    uint64_t next_block = 0, next_q = 0, consumed = 0;
    uint64_t limit_base = 0;  // device_bytes_cap
    // pending input on the device: double buffers, live bytes [head, tail)
    uint8_t* xbuf[2] = {nullptr, nullptr};
    uint8_t* ybuf[2] = {nullptr, nullptr};
    int xcur = 0, ycur = 0;
    uint64_t bcap = 0;
    uint64_t xhead = 0, xtail = 0, yhead = 0, ytail = 0;
    // outputs: byte ring; a call's outputs never wrap
    uint8_t* oring = nullptr;
    uint64_t ocap = 0;
    uint64_t owrite = 0, oread = 0;  // monotonic positions
    std::deque<GLaunch> inflight;
    uint64_t launched = 0, returned = 0;
    // device launch tables (queued calls run in stream order, so one set)
    uint8_t* dtab = nullptr;
    uint32_t* dheads = nullptr;
    // the tables packed in pinned, coherent host memory, read by the staging
    // kernel: two sets, each reused once the kernel that read it has run
    uint8_t* ptab = nullptr;
    hipEvent_t ptab_free[2] = {nullptr, nullptr};
    int ptab_next = 0;
    // pinned, coherent staging of host submissions (read by the staging kernel)
    uint8_t* stage = nullptr;
    uint64_t stage_bytes = 0;
    hipEvent_t stage_free = nullptr;
    // byte moves of the current submission (compaction, appended chunks),
    // run by the next staging kernel
    qext::CopySegs segs{};
    Planned plan;
};

namespace {

uint64_t block_bytes(const ext_growing_stream* s, uint64_t q) { return q * s->g->n_e / 8; }

// Blocks per queued call: a block has at most n_e slices, so the call's tiles
// stay within kMaxLaunchTiles.
uint64_t call_blocks(const ext_growing_stream* s) {
    return std::max<uint64_t>(1, std::min<uint64_t>(kMaxLaunchBlocks,
                                                    kMaxLaunchTiles / s->g->n_e));
}

// Admission limit on the pending bytes of one side: the cap, bounded so that
// their outputs (at most 1/n_e of them) fit in half the output ring, but
// never below two blocks of the next degree.
uint64_t limit_bytes(const ext_growing_stream* s) {
    const uint64_t by_ring = s->ocap / 2 * s->g->n_e;
    return std::max(std::min(s->limit_base, by_ring), 2 * block_bytes(s, s->next_q));
}

void free_stream(ext_growing_stream* s) {
    for (GLaunch& L : s->inflight)
        if (L.done) (void)hipEventDestroy(L.done);
    s->inflight.clear();
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(s->xbuf[k]);
        (void)hipFree(s->ybuf[k]);
        if (s->ptab_free[k]) (void)hipEventDestroy(s->ptab_free[k]);
    }
    (void)hipFree(s->oring);
    (void)hipFree(s->dtab);
    (void)hipFree(s->dheads);
    if (s->ptab) (void)hipHostFree(s->ptab);
    if (s->stage) (void)hipHostFree(s->stage);
    if (s->stage_free) (void)hipEventDestroy(s->stage_free);
    delete s;
}

int sfail(ext_growing_stream* s) {
    (void)hipGetLastError();
    return s->g->sticky = EXT_EDEVICE;
}

// Whole blocks that `avail` more bytes per source complete from the state
// (next_q), at most max_k; their input and output bytes.
void complete_blocks(const ext_growing_stream* s, uint64_t avail, uint64_t max_k, uint64_t* k,
                     uint64_t* in_bytes, uint64_t* out_bytes) {
    uint64_t q = s->next_q, n = 0, ib = 0, ob = 0;
    while (n < max_k) {
        const uint64_t nb = block_bytes(s, q);
        if (ib + nb > avail) break;
        ib += nb;
        ob += q / 8;
        ++n;
        q += s->step;
    }
    *k = n;
    *in_bytes = ib;
    *out_bytes = ob;
}

// The sequence of queued calls that k blocks from degree q0 make (at most
// call_blocks each), placed in the output ring from owrite: false if
// they do not fit beside the unreturned outputs.  sizes receives (k, bytes)
// per call and *end the ring position after the last.
bool ring_fit(const ext_growing_stream* s, uint64_t q0, uint64_t k,
              std::vector<std::pair<uint64_t, uint64_t>>* sizes, uint64_t* end) {
    uint64_t pos = s->owrite, q = q0;
    sizes->clear();
    while (k) {
        const uint64_t n = std::min(k, call_blocks(s));
        uint64_t ob = 0;
        for (uint64_t j = 0; j < n; ++j, q += s->step) ob += q / 8;
        if (ob > s->ocap) return false;
        const uint64_t off = pos % s->ocap;
        if (off + ob > s->ocap) pos += s->ocap - off;  // the call starts at the ring's front
        if (pos + ob - s->oread > s->ocap) return false;
        sizes->push_back({n, ob});
        pos += ob;
        k -= n;
    }
    *end = pos;
    return true;
}

void add_seg(ext_growing_stream* s, const uint8_t* src, uint8_t* dst, uint64_t len) {
    if (len) s->segs.seg[s->segs.n++] = qext::CopySeg{src, dst, len};
}

// Room for len more bytes after tail on one side: compact the live bytes to
// the front of the other buffer (a move of the next staging kernel), or grow
// both buffers (after waiting for the queued work that reads them).
int make_room(ext_growing_stream* s, uint8_t** buf, int* cur, uint64_t* head, uint64_t* tail,
              uint64_t len) {
    const uint64_t live = *tail - *head;
    if (*tail + len <= s->bcap) return EXT_OK;
    if (live + len <= s->bcap) {
        const int nxt = 1 - *cur;
        add_seg(s, buf[*cur] + *head, buf[nxt], live);
        *cur = nxt;
        *head = 0;
        *tail = live;
        return EXT_OK;
    }
    return EXT_EAGAIN;  // the caller grows the buffers first
}

// Grow the pending buffers to at least `need` bytes per buffer.
int grow_pending(ext_growing_stream* s, uint64_t need) {
    ext_growing* g = s->g;
    uint64_t cap = std::max<uint64_t>(2 * s->bcap, need);
    cap = (cap + 255) / 256 * 256;
    uint8_t* nx[2] = {nullptr, nullptr};
    uint8_t* ny[2] = {nullptr, nullptr};
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipMalloc((void**)&nx[k], cap) == hipSuccess &&
             hipMalloc((void**)&ny[k], cap) == hipSuccess;
    if (!ok) {
        for (int k = 0; k < 2; ++k) {
            (void)hipFree(nx[k]);
            (void)hipFree(ny[k]);
        }
        (void)hipGetLastError();
        return EXT_ENOMEM;
    }
    const uint64_t xl = s->xtail - s->xhead, yl = s->ytail - s->yhead;
    if ((xl && hipMemcpyAsync(nx[0], s->xbuf[s->xcur] + s->xhead, xl, hipMemcpyDeviceToDevice,
                              g->stream) != hipSuccess) ||
        (yl && hipMemcpyAsync(ny[0], s->ybuf[s->ycur] + s->yhead, yl, hipMemcpyDeviceToDevice,
                              g->stream) != hipSuccess) ||
        hipStreamSynchronize(g->stream) != hipSuccess) {
        for (int k = 0; k < 2; ++k) {
            (void)hipFree(nx[k]);
            (void)hipFree(ny[k]);
        }
        return sfail(s);
    }
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(s->xbuf[k]);
        (void)hipFree(s->ybuf[k]);
        s->xbuf[k] = nx[k];
        s->ybuf[k] = ny[k];
    }
    s->xcur = s->ycur = 0;
    s->xhead = s->yhead = 0;
    s->xtail = xl;
    s->ytail = yl;
    s->bcap = cap;
    return EXT_OK;
}

// The moves of one submission to the tails of the pending buffers, run by
// the next staging kernel: device data straight from the caller's memory,
// host data through pinned staging (reused once the previous staging kernel
// has run).
int append(ext_growing_stream* s, const void* x, uint64_t x_len, const void* y, uint64_t y_len) {
    ext_growing* g = s->g;
    uint8_t* xdst = s->xbuf[s->xcur] + s->xtail;
    uint8_t* ydst = s->ybuf[s->ycur] + s->ytail;
    if (g->params.mem_kind == EXT_MEM_DEVICE) {
        add_seg(s, (const uint8_t*)x, xdst, x_len);
        add_seg(s, (const uint8_t*)y, ydst, y_len);
        return EXT_OK;
    }
    if (!x_len && !y_len) return EXT_OK;
    if (hipEventSynchronize(s->stage_free) != hipSuccess) return sfail(s);
    const uint64_t len = x_len + y_len;
    if (s->stage_bytes < len) {
        if (s->stage) (void)hipHostFree(s->stage);
        s->stage = nullptr;
        s->stage_bytes = 0;
        if (hipHostMalloc((void**)&s->stage, len, hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return EXT_ENOMEM;
        }
        s->stage_bytes = len;
    }
    if (x_len) memcpy(s->stage, x, x_len);
    if (y_len) memcpy(s->stage + x_len, y, y_len);
    add_seg(s, s->stage, xdst, x_len);
    add_seg(s, s->stage + x_len, ydst, y_len);
    return EXT_OK;
}

// Queue the staging kernel on g->stream: the pending moves and, for a call,
// its packed tables (meta_bytes at meta_src, pinned) into s->dtab and n_heads
// cleared queue heads.  In host-memory mode the pinned staging is free again
// once this kernel has run.
int issue_stage(ext_growing_stream* s, const void* meta_src, uint32_t meta_bytes,
                uint32_t n_heads) {
    ext_growing* g = s->g;
    const bool host_moves = s->segs.n && g->params.mem_kind == EXT_MEM_HOST;
    const hipError_t e = qext::launch_copy_stage(s->segs, meta_src, s->dtab, meta_bytes,
                                                 s->dheads, n_heads, g->stream);
    s->segs.n = 0;
    if (e != hipSuccess) return sfail(s);
    if (host_moves && hipEventRecord(s->stage_free, g->stream) != hipSuccess) return sfail(s);
    return EXT_OK;
}

// Launch every block the pending bytes complete, in calls of at most
// call_blocks blocks placed as ring_fit placed them.
int launch_ready(ext_growing_stream* s) {
    ext_growing* g = s->g;
    uint64_t k, ib, ob;
    complete_blocks(s, std::min(s->xtail - s->xhead, s->ytail - s->yhead), ~0ull, &k, &ib, &ob);
    if (!k) return EXT_OK;
    std::vector<std::pair<uint64_t, uint64_t>> sizes;
    uint64_t end = 0;
    if (!ring_fit(s, s->next_q, k, &sizes, &end)) return EXT_EAGAIN;  // checked by the caller
    for (const auto& sz : sizes) {
        const uint64_t n = sz.first, bytes = sz.second;
        uint64_t pos = s->owrite;
        const uint64_t off = pos % s->ocap;
        if (off + bytes > s->ocap) pos += s->ocap - off;
        const uint8_t* xp = s->xbuf[s->xcur] + s->xhead;
        const uint8_t* yp = s->ybuf[s->ycur] + s->yhead;
        int rc = plan_blocks(g, s->next_q, n, xp, yp, s->oring + pos % s->ocap, true, &s->plan);
        if (rc) return rc;
        if (s->plan.tiles.size() > kMaxLaunchTiles) return EXT_ENOTSUP;
        rc = grow_part(g, s->plan.part_words);
        if (rc) return rc;
        // the pinned table set of the call before last is free once the
        // staging kernel that read it has run
        const int slot = s->ptab_next;
        if (hipEventSynchronize(s->ptab_free[slot]) != hipSuccess) return sfail(s);
        uint8_t* pt = s->ptab + slot * kTableBytes;
        const size_t sb = s->plan.streams.size() * sizeof(BatchStream);
        const size_t tb = s->plan.tiles.size() * sizeof(BatchTile);
        const size_t jb = s->plan.jobs.size() * sizeof(CombineJob);
        const size_t to = round16(sb), jo = to + round16(tb), total = jo + round16(jb);
        memcpy(pt, s->plan.streams.data(), sb);
        memcpy(pt + to, s->plan.tiles.data(), tb);
        memcpy(pt + jo, s->plan.jobs.data(), jb);
        const Tables tab{(BatchStream*)s->dtab, (BatchTile*)(s->dtab + to),
                         (CombineJob*)(s->dtab + jo), s->dheads};
        // the submission's moves ride with the first call's tables
        rc = issue_stage(s, pt, (uint32_t)total, (uint32_t)s->plan.launches.size());
        if (rc) return rc;
        if (hipEventRecord(s->ptab_free[slot], g->stream) != hipSuccess) return sfail(s);
        s->ptab_next = 1 - slot;
        rc = queue_launches(g, s->plan, tab);
        if (rc) return rc;
        GLaunch L{s->next_block, n, s->next_q, pos, bytes};
        if (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess)
            return sfail(s);
        if (hipEventRecord(L.done, g->stream) != hipSuccess) {
            (void)hipEventDestroy(L.done);
            return sfail(s);
        }
        s->inflight.push_back(L);
        s->owrite = pos + bytes;
        uint64_t in = 0;
        for (uint64_t j = 0; j < n; ++j) {
            in += block_bytes(s, s->next_q);
            s->next_q += s->step;
        }
        s->next_block += n;
        s->consumed += in;
        s->launched += n;
        s->xhead += in;
        s->yhead += in;
    }
    return EXT_OK;
}

// Copy whole finished blocks into out, in block order: the ring ranges of
// consecutive blocks are merged into as few copies as possible.  Device
// memory on the caller's HIP stream: the copies are queued on it (later work
// there, including this stream's next launches, comes after them); else they
// run on g->copy and are waited for once before returning (drain always
// waits).
int copy_out(ext_growing_stream* s, void* out, size_t out_cap, size_t* out_len,
             uint64_t* blocks_done, bool wait) {
    ext_growing* g = s->g;
    const bool device = g->params.mem_kind == EXT_MEM_DEVICE;
    const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const bool ordered = device && g->params.use_hip_stream;
    hipStream_t cs = ordered ? g->stream : g->copy;
    size_t written = 0;
    uint64_t run_src = 0, run_len = 0;  // the copy being merged: ring offset, bytes
    size_t run_dst = 0;
    auto flush = [&]() {
        const bool ok = !run_len || hipMemcpyAsync((uint8_t*)out + run_dst, s->oring + run_src,
                                                   run_len, kind, cs) == hipSuccess;
        run_len = 0;
        return ok;
    };
    while (!s->inflight.empty()) {
        GLaunch& L = s->inflight.front();
        if (wait) {
            if (hipEventSynchronize(L.done) != hipSuccess) return sfail(s);
        } else {
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return sfail(s);
        }
        // whole blocks that fit
        uint64_t n = 0, bytes = 0;
        uint64_t q = L.q0 + L.taken * s->step;
        while (L.taken + n < L.k && written + bytes + q / 8 <= out_cap) {
            bytes += q / 8;
            ++n;
            q += s->step;
        }
        if (n) {
            const uint64_t src = (L.opos + L.taken_bytes) % s->ocap;
            if (run_len && src == run_src + run_len) {
                run_len += bytes;
            } else {
                if (!flush()) return sfail(s);
                run_src = src;
                run_dst = written;
                run_len = bytes;
            }
            written += bytes;
            L.taken += n;
            L.taken_bytes += bytes;
            s->returned += n;
        }
        if (L.taken < L.k) break;  // the caller's buffer is full
        s->oread = L.opos + L.obytes;
        (void)hipEventDestroy(L.done);
        s->inflight.pop_front();
    }
    // the ring ranges handed back may be overwritten by later launches only
    // after these copies: stream order, or a wait before returning
    if (!flush() || (written && (!ordered || wait) && hipStreamSynchronize(cs) != hipSuccess))
        return sfail(s);
    if (out_len) *out_len = written;
    if (blocks_done) *blocks_done = s->returned;
    return EXT_OK;
}

int genter(ext_growing_stream* s) {
    if (!s) return EXT_EINVAL;
    if (s->g->sticky) return s->g->sticky;
    if (hipSetDevice(s->g->device) != hipSuccess) return EXT_EDEVICE;
    return EXT_OK;
}

}  // namespace

extern "C" {

int ext_growing_open(ext_growing* g, ext_growing_stream** out) {
    if (!g || !out) return EXT_EINVAL;
    *out = nullptr;
    if (g->sticky) return g->sticky;
    if (hipSetDevice(g->device) != hipSuccess) return EXT_EDEVICE;
    ext_growing_stream* s = new (std::nothrow) ext_growing_stream;
    if (!s) return EXT_ENOMEM;
    s->g = g;
    s->step = (uint64_t)g->delta_steps * g->b;
    s->next_q = g->q1;
    s->limit_base = g->params.device_bytes_cap ? g->params.device_bytes_cap : (256ull << 20);
    // pending bytes: room for a few first blocks, grown on demand
    s->bcap = std::max<uint64_t>(1ull << 20, 4 * block_bytes(s, g->q1));
    s->bcap = (s->bcap + 255) / 256 * 256;
    // outputs: twice what the admitted pending input can complete
    s->ocap = std::min<uint64_t>(64ull << 20,
                                 std::max<uint64_t>(1ull << 20, 2 * s->limit_base / g->n_e));
    s->ocap = (s->ocap + 255) / 256 * 256;
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipMalloc((void**)&s->xbuf[k], s->bcap) == hipSuccess &&
             hipMalloc((void**)&s->ybuf[k], s->bcap) == hipSuccess &&
             hipEventCreateWithFlags(&s->ptab_free[k], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->oring, s->ocap) == hipSuccess &&
         hipMalloc((void**)&s->dtab, kTableBytes) == hipSuccess &&
         hipMalloc((void**)&s->dheads, kMaxGroups * sizeof(uint32_t)) == hipSuccess &&
         hipHostMalloc((void**)&s->ptab, 2 * kTableBytes, hipHostMallocCoherent) == hipSuccess &&
         hipEventCreateWithFlags(&s->stage_free, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_stream(s);
        return EXT_ENOMEM;
    }
    try {
        g->open_streams.push_back(s);
    } catch (const std::bad_alloc&) {
        free_stream(s);
        return EXT_ENOMEM;
    }
    *out = s;
    return EXT_OK;
}

int ext_growing_submit(ext_growing_stream* s, const void* x, size_t x_len, const void* y,
                       size_t y_len, uint64_t* blocks_launched) {
    int rc = genter(s);
    if (rc) return rc;
    if ((x_len && !x) || (y_len && !y)) return EXT_EINVAL;
    const uint64_t xl = s->xtail - s->xhead, yl = s->ytail - s->yhead;
    // admission: pending bytes per side within the limit
    const uint64_t lim = limit_bytes(s);
    if (xl + x_len > lim || yl + y_len > lim) return EXT_EAGAIN;
    try {
        // the blocks this chunk completes: every degree planned (so a degree
        // without modulus or plan refuses the chunk whole), outputs placed
        uint64_t k, ib, ob;
        complete_blocks(s, std::min(xl + x_len, yl + y_len), ~0ull, &k, &ib, &ob);
        uint64_t q = s->next_q;
        for (uint64_t j = 0; j < k; ++j, q += s->step) {
            DegreePlan d;
            if (q > 0xffffffffull) return EXT_ENOTSUP;
            rc = plan_for(s->g, (uint32_t)q, &d);
            if (rc) return rc;
        }
        std::vector<std::pair<uint64_t, uint64_t>> sizes;
        uint64_t end = 0;
        if (k && !ring_fit(s, s->next_q, k, &sizes, &end)) return EXT_EAGAIN;
        const uint64_t need = std::max(xl + x_len, yl + y_len);
        if (need > s->bcap) {
            rc = grow_pending(s, need);
            if (rc) return rc;
        }
        // moves (compaction, the chunks), then the blocks completed; moves not
        // carried by a call's staging kernel (none completed, or an error
        // after a compaction switched buffers) go in one of their own
        rc = make_room(s, s->xbuf, &s->xcur, &s->xhead, &s->xtail, x_len);
        if (!rc) rc = make_room(s, s->ybuf, &s->ycur, &s->yhead, &s->ytail, y_len);
        if (!rc) rc = append(s, x, x_len, y, y_len);
        if (!rc) {
            s->xtail += x_len;
            s->ytail += y_len;
            rc = launch_ready(s);
        }
        if (s->segs.n) {
            const int rc2 = issue_stage(s, nullptr, 0, 0);
            if (!rc) rc = rc2;
        }
        if (rc) return rc;
    } catch (const std::bad_alloc&) {
        return EXT_ENOMEM;
    }
    if (blocks_launched) *blocks_launched = s->launched;
    return EXT_OK;
}

int ext_growing_poll(ext_growing_stream* s, void* out, size_t out_cap, size_t* out_len,
                     uint64_t* blocks_done) {
    const int rc = genter(s);
    if (rc) return rc;
    if (!out && out_cap) return EXT_EINVAL;
    return copy_out(s, out, out_cap, out_len, blocks_done, false);
}

int ext_growing_drain(ext_growing_stream* s, void* out, size_t out_cap, size_t* out_len,
                      uint64_t* blocks_done) {
    const int rc = genter(s);
    if (rc) return rc;
    if (!out && out_cap) return EXT_EINVAL;
    return copy_out(s, out, out_cap, out_len, blocks_done, true);
}

int ext_growing_state(const ext_growing_stream* s, uint64_t* next_block, uint64_t* next_q,
                      uint64_t* consumed_bytes) {
    if (!s) return EXT_EINVAL;
    if (next_block) *next_block = s->next_block;
    if (next_q) *next_q = s->next_q;
    if (consumed_bytes) *consumed_bytes = s->consumed;
    return EXT_OK;
}

int ext_growing_close(ext_growing_stream* s, uint64_t* dropped_bits) {
    if (!s) return EXT_EINVAL;
    ext_growing* g = s->g;
    const uint64_t px = s->xtail - s->xhead, py = s->ytail - s->yhead;
    if (dropped_bits) *dropped_bits = 8 * std::max(px, py);
    (void)hipSetDevice(g->device);
    (void)hipStreamSynchronize(g->stream);
    auto it = std::find(g->open_streams.begin(), g->open_streams.end(), s);
    if (it != g->open_streams.end()) g->open_streams.erase(it);
    free_stream(s);
    return EXT_OK;
}

}  // extern "C"
