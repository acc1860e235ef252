// ext_batch.cpp -- batched form (many streams of different shapes in one
// persistent launch fed by a device work queue, captured in a hipGraph) and
// the autotuner that picks each shape's launch plan by timing candidates.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <random>
#include <tuple>
#include <vector>

#include "../../include/qrng_ext.h"
#include "ext_internal.h"
#include "gf2_modulus.h"

namespace qext {

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

struct TuneKey {
    int device;
    uint32_t q, n_e, n_taps, t0, t1, t2;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, q, n_e, n_taps, t0, t1, t2) <
               std::tie(o.device, o.q, o.n_e, o.n_taps, o.t0, o.t1, o.t2);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, std::pair<PlanKnobs, float>> g_tune_cache;

}  // namespace

// Time every candidate plan of (q, n_e, taps) on `stream` over synthetic
// blocks and return the fastest.  Candidates: base sizes of 128, 256 and 512
// bits, every element grouping, the planner's pairs per work-group, and
// 1024-lane work-groups for shapes with more than 256 items per pair.
hipError_t autotune_shape(uint32_t q, uint32_t n_e, const uint32_t* taps, uint32_t n_taps,
                          hipStream_t stream, PlanKnobs* best, float* best_ms) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    TuneKey key{dev, q, n_e, n_taps, n_taps > 0 ? taps[0] : 0, n_taps > 1 ? taps[1] : 0,
                n_taps > 2 ? taps[2] : 0};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return hipSuccess;
        }
    }
    std::vector<std::pair<PlanKnobs, ExtShape>> cands;
    for (uint32_t nt : {(uint32_t)kThreads, (uint32_t)kMaxThreads})
    for (uint32_t bwt : {4u, 8u, 16u})
        for (uint32_t g = 1; g <= n_e; ++g) {
            // (plan_shape rejects a group count that ceil-sized groups do not realise)
            PlanKnobs k{bwt, g, 0, nt};
            ExtShape s;
            if (!plan_shape(q, n_e, taps, n_taps, k, &s)) continue;
            // wide groups only where one pair has more items than a narrow group has lanes
            if (nt != (uint32_t)kThreads && (uint64_t)s.np * s.groups <= (uint64_t)kThreads) continue;
            bool dup = false;
            for (auto& c : cands)
                dup |= c.second.bw == s.bw && c.second.groups == s.groups && c.second.ppw == s.ppw &&
                       c.second.threads == s.threads;
            if (!dup) cands.push_back({PlanKnobs{s.bw, s.groups, s.ppw, s.threads}, s});
        }
    if (cands.empty()) return hipErrorInvalidValue;

    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // enough pairs for ~8 work-groups per CU with the largest ppw, capped at 64 MiB
    uint32_t max_ppw = 1;
    for (auto& c : cands) max_ppw = std::max(max_ppw, c.second.ppw);
    const uint64_t nb = (uint64_t)q * n_e / 8;
    uint64_t pairs = (uint64_t)cus * 8 * max_ppw;
    pairs = std::max<uint64_t>(1, std::min<uint64_t>(pairs, (64ull << 20) / nb));
    uint8_t *dx = nullptr, *dy = nullptr, *dout = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<uint8_t> host(pairs * nb);
    std::mt19937_64 rng(0x5eed ^ q ^ (uint64_t)n_e << 32);
    for (auto& b : host) b = (uint8_t)rng();
    float best_t = 1e30f;
    size_t best_i = 0;
    do {
        if ((e = hipMalloc((void**)&dx, pairs * nb)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&dy, pairs * nb)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&dout, pairs * q / 8)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(dx, host.data(), pairs * nb, hipMemcpyHostToDevice, stream)) !=
            hipSuccess)
            break;
        if ((e = hipMemcpyAsync(dy, host.data(), pairs * nb, hipMemcpyHostToDevice, stream)) !=
            hipSuccess)
            break;
        if ((e = hipEventCreate(&e0)) != hipSuccess) break;
        if ((e = hipEventCreate(&e1)) != hipSuccess) break;
        for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
            const ExtShape& s = cands[i].second;
            auto run = [&] {
                return launch_extract(s, (const uint8_t*)dx, (const uint8_t*)dy, (uint8_t*)dout,
                                      pairs, stream);
            };
            if ((e = run()) != hipSuccess) break;
            if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
            if (e != hipSuccess) break;
            if ((e = hipEventRecord(e1, stream)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            // normalise to time per pair
            const float per = ms / 3.0f / (float)pairs;
            if (per < best_t) {
                best_t = per;
                best_i = i;
            }
        }
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dx);
    (void)hipFree(dy);
    (void)hipFree(dout);
    if (e != hipSuccess) return e;
    *best = cands[best_i].first;
    if (best_ms) *best_ms = best_t;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = {*best, best_t};
    return hipSuccess;
}

namespace {
std::map<TuneKey, bool> g_kernel_cache;
}  // namespace

// Word-level plan (tuned by autotune_shape) against the bit-sliced kernel:
// time per pair of each over synthetic blocks, the faster one wins.
hipError_t choose_kernel(const ExtShape& bs, hipStream_t stream, bool* use_bitslice) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const TuneKey key{dev, bs.q, bs.n_e, bs.n_taps, bs.n_taps > 0 ? bs.taps[0] : 0,
                      bs.n_taps > 1 ? bs.taps[1] : 0, bs.n_taps > 2 ? bs.taps[2] : 0};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_kernel_cache.find(key);
        if (it != g_kernel_cache.end()) {
            *use_bitslice = it->second;
            return hipSuccess;
        }
    }
    PlanKnobs knobs;
    float word_per_pair = 0;
    e = autotune_shape(bs.q, bs.n_e, bs.taps, bs.n_taps, stream, &knobs, &word_per_pair);
    if (e != hipSuccess) return e;
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const uint64_t nb = bs.nbytes;
    uint64_t pairs = (uint64_t)cus * 8 * 32;  // ~8 work-groups of 32 pairs per CU
    pairs = std::max<uint64_t>(32, std::min<uint64_t>(pairs, (64ull << 20) / nb));
    uint8_t *dx = nullptr, *dy = nullptr, *dout = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<uint8_t> host(pairs * nb);
    std::mt19937_64 rng(0x5eed ^ bs.q ^ (uint64_t)bs.n_e << 32);
    for (auto& b : host) b = (uint8_t)rng();
    float bs_per_pair = 1e30f;
    do {
        if ((e = hipMalloc((void**)&dx, pairs * nb)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&dy, pairs * nb)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&dout, pairs * bs.qbytes)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(dx, host.data(), pairs * nb, hipMemcpyHostToDevice, stream)) !=
            hipSuccess)
            break;
        if ((e = hipMemcpyAsync(dy, host.data(), pairs * nb, hipMemcpyHostToDevice, stream)) !=
            hipSuccess)
            break;
        if ((e = hipEventCreate(&e0)) != hipSuccess) break;
        if ((e = hipEventCreate(&e1)) != hipSuccess) break;
        auto run = [&] { return launch_bitslice(bs, dx, dy, dout, pairs, stream); };
        if ((e = run()) != hipSuccess) break;
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
        if (e != hipSuccess) break;
        if ((e = hipEventRecord(e1, stream)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        bs_per_pair = ms / 3.0f / (float)pairs;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dx);
    (void)hipFree(dy);
    (void)hipFree(dout);
    if (e != hipSuccess) return e;
    *use_bitslice = bs_per_pair < word_per_pair;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_kernel_cache[key] = *use_bitslice;
    return hipSuccess;
}

}  // namespace qext

// ---------------------------------------------------------------------------
// batch object
// ---------------------------------------------------------------------------
using qext::BatchStream;
using qext::BatchTile;
using qext::ExtShape;

struct ext_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    struct Group {
        uint32_t bw, threads, padded, tile_off, n_tiles, lds_bytes, grid;
    };
    std::vector<Group> groups;
    std::vector<BatchStream> streams;  // host copy (device pointers inside)
    std::vector<BatchTile> tiles;
    BatchStream* d_streams = nullptr;
    BatchTile* d_tiles = nullptr;
    uint32_t* d_heads = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t total_pairs = 0;
    double total_bitmacs = 0;
    int sticky = EXT_OK;
};

namespace {

void batch_free(ext_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_streams);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_heads);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int enqueue(ext_batch* b) {
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const auto& g = b->groups[gi];
        hipError_t e = qext::launch_batch(g.bw, g.threads, g.padded != 0, b->d_streams,
                                          b->d_tiles + g.tile_off,
                                          g.n_tiles,
                                          b->d_heads + gi, g.grid, g.lds_bytes, b->stream);
        if (e != hipSuccess) return EXT_EDEVICE;
    }
    return EXT_OK;
}

}  // namespace

extern "C" {

int ext_batch_create(const ext_batch_item* items, uint32_t n_items, const ext_params* p,
                     ext_batch** out) {
    if (!out || (n_items && !items)) return EXT_EINVAL;
    *out = nullptr;
    ext_params def;
    ext_params_init(&def);
    if (!p) p = &def;
    if (p->n_taps) return EXT_EINVAL;  // batches use the conventional modulus of each m
    if (p->kernel > EXT_KERNEL_BITSLICE) return EXT_EINVAL;
    if (p->kernel == EXT_KERNEL_BITSLICE) return EXT_ENOTSUP;  // word-level kernels only
    ext_batch* b = new (std::nothrow) ext_batch;
    if (!b) return EXT_ENOMEM;
    int dev = p->device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        delete b;
        return EXT_EDEVICE;
    }
    b->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
        delete b;
        return EXT_EDEVICE;
    }
    // graph capture needs a stream other than the legacy null stream
    if (p->use_hip_stream && p->hip_stream) {
        b->stream = (hipStream_t)p->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return EXT_EDEVICE;
        }
        b->own_stream = true;
    }
    int rc = EXT_OK;
    try {
        // plan every stream
        // launches: one per (base size, work-group size, padded) -> stream indices
        std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::vector<uint32_t>> by_bw;
        for (uint32_t i = 0; i < n_items && rc == EXT_OK; ++i) {
            const ext_batch_item& it = items[i];
            if (it.n_bits == 0 || it.m_bits == 0 || it.n_bits % it.m_bits ||
                it.n_bits / it.m_bits > 0xffffffffull || (it.n_pairs && (!it.x || !it.y || !it.out))) {
                rc = EXT_EINVAL;
                break;
            }
            std::vector<uint32_t> taps;
            if (!qext::default_modulus(it.m_bits, &taps)) {
                rc = EXT_ENOTSUP;
                break;
            }
            const uint32_t n_e = (uint32_t)(it.n_bits / it.m_bits);
            qext::PlanKnobs knobs{p->base_bits / 32, p->groups, p->pairs_per_group, p->threads};
            if (p->autotune) {
                if (qext::autotune_shape(it.m_bits, n_e, taps.data(), (uint32_t)taps.size(),
                                         b->stream, &knobs, nullptr) != hipSuccess) {
                    rc = EXT_EDEVICE;
                    break;
                }
            }
            ExtShape s;
            if (!qext::plan_shape(it.m_bits, n_e, taps.data(), (uint32_t)taps.size(), knobs, &s)) {
                rc = EXT_ENOTSUP;
                break;
            }
            const uintptr_t am = s.align - 1;
            if (((uintptr_t)it.x & am) || ((uintptr_t)it.y & am) || ((uintptr_t)it.out & 3)) {
                rc = EXT_EINVAL;
                break;
            }
            BatchStream st{(const uint8_t*)it.x, (const uint8_t*)it.y, (uint8_t*)it.out,
                           it.n_pairs, s};
            b->streams.push_back(st);
            by_bw[std::make_tuple(s.bw, s.threads, s.padded)].push_back(i);
            b->total_pairs += it.n_pairs;
            b->total_bitmacs += (double)it.n_pairs * (double)it.n_bits * (double)it.m_bits;
        }
        if (rc == EXT_OK) {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess)
                rc = EXT_EDEVICE;
            for (auto& kv : by_bw) {
                if (rc != EXT_OK) break;
                ext_batch::Group g{std::get<0>(kv.first), std::get<1>(kv.first),
                                   std::get<2>(kv.first), (uint32_t)b->tiles.size(), 0, 0, 0};
                std::vector<std::pair<double, BatchTile>> tl;
                for (uint32_t si : kv.second) {
                    const BatchStream& st = b->streams[si];
                    g.lds_bytes = std::max(g.lds_bytes, st.shape.lds_words * 4);
                    // cost of one tile ~ base products per lane-slot it occupies
                    const double per_pair = (double)st.shape.np * st.shape.n_e;
                    for (uint64_t p0 = 0; p0 < st.n_pairs; p0 += st.shape.ppw) {
                        const uint32_t k = (uint32_t)std::min<uint64_t>(st.shape.ppw, st.n_pairs - p0);
                        tl.push_back({per_pair * k, BatchTile{si, k, p0, p0 * st.shape.qbytes, 0, 0}});
                    }
                }
                // longest tiles first, so the queue ends with short ones
                std::stable_sort(tl.begin(), tl.end(),
                                 [](const auto& a, const auto& c) { return a.first > c.first; });
                for (auto& t : tl) b->tiles.push_back(t.second);
                g.n_tiles = (uint32_t)tl.size();
                int occ = 0;
                if (qext::batch_occupancy(g.bw, g.threads, g.padded != 0, g.lds_bytes, &occ) !=
                        hipSuccess ||
                    occ <= 0)
                    occ = 1;
                g.grid = (uint32_t)std::min<uint64_t>(g.n_tiles, (uint64_t)cus * occ);
                if (g.n_tiles) b->groups.push_back(g);
            }
        }
    } catch (const std::bad_alloc&) {
        rc = EXT_ENOMEM;
    }
    if (rc != EXT_OK) {
        batch_free(b);
        return rc;
    }
    bool ok = true;
    if (!b->streams.empty())
        ok = hipMalloc((void**)&b->d_streams, b->streams.size() * sizeof(BatchStream)) == hipSuccess &&
             hipMemcpy(b->d_streams, b->streams.data(), b->streams.size() * sizeof(BatchStream),
                       hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !b->tiles.empty())
        ok = hipMalloc((void**)&b->d_tiles, b->tiles.size() * sizeof(BatchTile)) == hipSuccess &&
             hipMemcpy(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(BatchTile),
                       hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !b->groups.empty())
        ok = hipMalloc((void**)&b->d_heads, b->groups.size() * sizeof(uint32_t)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        batch_free(b);
        return EXT_ENOMEM;
    }
    // capture the submission once; ext_batch_run replays it
    if (!b->groups.empty()) {
        bool captured =
            hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (captured) {
            const int erc = enqueue(b);
            captured = hipStreamEndCapture(b->stream, &b->graph) == hipSuccess && erc == EXT_OK;
        }
        if (captured)
            captured = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
        if (!captured) {
            (void)hipGetLastError();
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
            b->exec = nullptr;
        }
    }
    *out = b;
    return EXT_OK;
}

int ext_batch_run(ext_batch* b) {
    if (!b) return EXT_EINVAL;
    if (b->sticky) return b->sticky;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || (cur != b->device && hipSetDevice(b->device) != hipSuccess))
        return b->sticky = EXT_EDEVICE;
    if (b->groups.empty()) return EXT_OK;
    if (b->exec) {
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return b->sticky = EXT_EDEVICE;
        return EXT_OK;
    }
    const int rc = enqueue(b);
    if (rc) b->sticky = rc;
    return rc;
}

int ext_batch_sync(ext_batch* b) {
    if (!b) return EXT_EINVAL;
    if (b->sticky) return b->sticky;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return b->sticky = EXT_EDEVICE;
    return EXT_OK;
}

int ext_batch_describe(const ext_batch* b, char* buf, size_t cap) {
    if (!b || !buf || !cap) return EXT_EINVAL;
    size_t n = (size_t)snprintf(buf, cap,
                                "{\"streams\": %zu, \"tiles\": %zu, \"pairs\": %llu, "
                                "\"bitmacs\": %.6e, \"graph\": %s, \"launches\": [",
                                b->streams.size(), b->tiles.size(),
                                (unsigned long long)b->total_pairs, b->total_bitmacs,
                                b->exec ? "true" : "false");
    for (size_t i = 0; i < b->groups.size() && n < cap; ++i) {
        const auto& g = b->groups[i];
        n += (size_t)snprintf(buf + n, cap - n,
                              "%s{\"base_bits\": %u, \"threads\": %u, \"padded\": %u, "
                              "\"tiles\": %u, \"grid\": %u, \"lds_bytes\": %u}",
                              i ? ", " : "", g.bw * 32, g.threads, g.padded, g.n_tiles, g.grid,
                              g.lds_bytes);
    }
    if (n < cap) snprintf(buf + n, cap - n, "]}");
    return EXT_OK;
}

int ext_batch_destroy(ext_batch* b) {
    if (!b) return EXT_OK;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != b->device) (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return EXT_OK;
}

}  // extern "C"
