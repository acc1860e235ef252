// ext_batch.cpp -- batched form (many streams of different shapes in one
// persistent launch fed by a device work queue, captured in a hipGraph) and
// the autotuner that picks each shape's launch plan by timing candidates.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <random>
#include <string>
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
std::map<TuneKey, bool> g_kernel_cache;

// ---- persisted results --------------------------------------------------
// The tuner's results outlive the process in a JSON file: an array with one
// object per line, either a plan ("entry": "plan": the knobs and the time
// per pair) or a kernel choice ("entry": "kernel": 1 = bit-sliced), keyed by
// the device ("gfx950:256": architecture and compute units), q, n_e and the
// modulus.  The file is $QRNG_EXT_TUNE_CACHE, else
// $XDG_CACHE_HOME/qrng_ext/autotune.json, else ~/.cache/qrng_ext/autotune.json;
// an empty QRNG_EXT_TUNE_CACHE turns persistence off.  It is read when a
// device first looks a shape up and rewritten (temporary file + rename)
// after every new timing; concurrent writers: the last one wins.
struct TuneEntry {
    std::string dev;
    uint32_t q, n_e, n_taps, t[3];
    bool plan;  // else a kernel choice
    PlanKnobs knobs;
    float ms;
    bool bitslice;
};
std::vector<TuneEntry> g_file;  // the file's entries (and ours since)
std::string g_file_path;
bool g_file_read = false;
std::map<int, std::string> g_dev_tags;

std::string tune_cache_path() {
    const char* e = getenv("QRNG_EXT_TUNE_CACHE");
    if (e) return std::string(e);
    const char* x = getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/qrng_ext/autotune.json";
    const char* h = getenv("HOME");
    if (h && *h) return std::string(h) + "/.cache/qrng_ext/autotune.json";
    return std::string();
}

std::string device_tag(int dev) {
    auto it = g_dev_tags.find(dev);
    if (it != g_dev_tags.end()) return it->second;
    hipDeviceProp_t prop;
    std::string tag = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string arch(prop.gcnArchName);
        const size_t colon = arch.find(':');  // drop feature suffixes (":sramecc+:xnack-")
        if (colon != std::string::npos) arch = arch.substr(0, colon);
        tag = arch + ":" + std::to_string(prop.multiProcessorCount);
    } else {
        (void)hipGetLastError();
    }
    g_dev_tags[dev] = tag;
    return tag;
}

// (lock held) read the file once per path
void read_tune_file() {
    const std::string path = tune_cache_path();
    if (g_file_read && path == g_file_path) return;
    g_file_read = true;
    g_file_path = path;
    g_file.clear();
    if (path.empty()) return;
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        TuneEntry t{};
        char dev[64] = {0}, kind[16] = {0};
        int used = 0;
        if (sscanf(line,
                   " {\"device\": \"%63[^\"]\", \"q\": %u, \"n_e\": %u, \"n_taps\": %u, "
                   "\"taps\": [%u, %u, %u], \"entry\": \"%15[^\"]\",%n",
                   dev, &t.q, &t.n_e, &t.n_taps, &t.t[0], &t.t[1], &t.t[2], kind, &used) != 8 ||
            t.n_taps > 3)
            continue;
        t.dev = dev;
        const char* rest = line + used;
        if (!strcmp(kind, "plan")) {
            t.plan = true;
            if (sscanf(rest, " \"base_words\": %u, \"groups\": %u, \"ppw\": %u, \"threads\": %u, "
                             "\"ms_per_pair\": %g",
                       &t.knobs.base_words, &t.knobs.groups, &t.knobs.ppw, &t.knobs.threads,
                       &t.ms) != 5)
                continue;
        } else if (!strcmp(kind, "kernel")) {
            unsigned v = 0;
            if (sscanf(rest, " \"bitslice\": %u", &v) != 1) continue;
            t.plan = false;
            t.bitslice = v != 0;
        } else {
            continue;
        }
        g_file.push_back(t);
    }
    fclose(f);
}

// (lock held) rewrite the file with every entry
void write_tune_file() {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    // create the directory (one level is enough for the default paths'
    // qrng_ext folder; ~/.cache itself normally exists)
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        const std::string dir = path.substr(0, slash);
        (void)mkdir(dir.c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "[\n");
    for (size_t i = 0; i < g_file.size(); ++i) {
        const TuneEntry& t = g_file[i];
        fprintf(f,
                "{\"device\": \"%s\", \"q\": %u, \"n_e\": %u, \"n_taps\": %u, "
                "\"taps\": [%u, %u, %u], \"entry\": \"%s\", ",
                t.dev.c_str(), t.q, t.n_e, t.n_taps, t.t[0], t.t[1], t.t[2],
                t.plan ? "plan" : "kernel");
        if (t.plan)
            fprintf(f,
                    "\"base_words\": %u, \"groups\": %u, \"ppw\": %u, \"threads\": %u, "
                    "\"ms_per_pair\": %.6g}",
                    t.knobs.base_words, t.knobs.groups, t.knobs.ppw, t.knobs.threads, t.ms);
        else
            fprintf(f, "\"bitslice\": %u}", t.bitslice ? 1u : 0u);
        fprintf(f, "%s\n", i + 1 < g_file.size() ? "," : "");
    }
    fprintf(f, "]\n");
    const bool ok = fclose(f) == 0;
    if (ok) (void)rename(tmp.c_str(), path.c_str());
    else (void)remove(tmp.c_str());
}

// (lock held) the file's entry for key (plan or kernel choice), if any
const TuneEntry* find_tune_entry(const TuneKey& key, bool plan) {
    read_tune_file();
    const std::string tag = device_tag(key.device);
    for (const TuneEntry& t : g_file)
        if (t.plan == plan && t.dev == tag && t.q == key.q && t.n_e == key.n_e &&
            t.n_taps == key.n_taps && t.t[0] == key.t0 && t.t[1] == key.t1 && t.t[2] == key.t2)
            return &t;
    return nullptr;
}

// (lock held) record a new result and rewrite the file
void add_tune_entry(const TuneKey& key, bool plan, const PlanKnobs& knobs, float ms,
                    bool bitslice) {
    read_tune_file();
    TuneEntry t{};
    t.dev = device_tag(key.device);
    t.q = key.q;
    t.n_e = key.n_e;
    t.n_taps = key.n_taps;
    t.t[0] = key.t0;
    t.t[1] = key.t1;
    t.t[2] = key.t2;
    t.plan = plan;
    t.knobs = knobs;
    t.ms = ms;
    t.bitslice = bitslice;
    g_file.push_back(t);
    write_tune_file();
}

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
        if (it == g_tune_cache.end()) {
            const TuneEntry* t = find_tune_entry(key, true);
            ExtShape chk;
            if (t && plan_shape(q, n_e, taps, n_taps, t->knobs, &chk))
                it = g_tune_cache.emplace(key, std::make_pair(t->knobs, t->ms)).first;
        }
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
    add_tune_entry(key, true, *best, best_t, false);
    return hipSuccess;
}

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
        if (it == g_kernel_cache.end()) {
            const TuneEntry* t = find_tune_entry(key, false);
            if (t) it = g_kernel_cache.emplace(key, t->bitslice).first;
        }
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
    add_tune_entry(key, false, PlanKnobs{}, 0.f, *use_bitslice);
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
    // the launches (one per base size) run concurrently: launch 0 on stream,
    // the others on side streams forked from and joined back into it, so that
    // each one's drain tail overlaps the next one's work
    static constexpr int kSides = 7;
    hipStream_t side[kSides] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSides] = {};
    uint64_t total_pairs = 0;
    double total_bitmacs = 0;
    int sticky = EXT_OK;
};

namespace {

void batch_free(ext_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int i = 0; i < ext_batch::kSides; ++i) {
        if (b->side[i]) {
            (void)hipStreamSynchronize(b->side[i]);
            (void)hipStreamDestroy(b->side[i]);
        }
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    (void)hipFree(b->d_streams);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_heads);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int enqueue(ext_batch* b) {
    const size_t n = b->groups.size();
    // fork: launch gi > 0 runs on side stream (gi - 1) % kSides after the
    // work queued on stream so far; join: stream waits for every side
    const bool forked = n > 1 && b->fork;
    if (forked && hipEventRecord(b->fork, b->stream) != hipSuccess) return EXT_EDEVICE;
    bool used[ext_batch::kSides] = {};
    for (size_t gi = 0; gi < n; ++gi) {
        const auto& g = b->groups[gi];
        hipStream_t st = b->stream;
        if (forked && gi > 0) {
            const int k = (int)((gi - 1) % ext_batch::kSides);
            st = b->side[k];
            if (!used[k] && hipStreamWaitEvent(st, b->fork, 0) != hipSuccess) return EXT_EDEVICE;
            used[k] = true;
        }
        hipError_t e = qext::launch_batch(g.bw, g.threads, g.padded != 0, b->d_streams,
                                          b->d_tiles + g.tile_off,
                                          g.n_tiles,
                                          b->d_heads + gi, g.grid, g.lds_bytes, st);
        if (e != hipSuccess) return EXT_EDEVICE;
    }
    for (int k = 0; k < ext_batch::kSides; ++k) {
        if (!used[k]) continue;
        if (hipEventRecord(b->join[k], b->side[k]) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->join[k], 0) != hipSuccess)
            return EXT_EDEVICE;
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
                    g.lds_bytes = std::max(g.lds_bytes, qext::group_lds_bytes(st.shape));
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
    if (b->groups.size() > 1) {
        bool sides = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
        for (int k = 0; sides && k < ext_batch::kSides; ++k)
            sides = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
                    hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
        if (!sides) {
            (void)hipGetLastError();
            batch_free(b);
            return EXT_EDEVICE;
        }
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
