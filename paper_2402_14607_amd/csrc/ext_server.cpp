// ext_server.cpp -- served form: continuous batching of many generator
// channels (each an (X, Y) pair of sample streams with its own block length).
//
// Data path, per cycle of the scheduler thread:
//   submit() copies raw chunks into the cycle's pinned staging area and notes
//   where each byte range goes in its channel's device ring (X and Y rings of
//   R blocks each; block l lives in slot l mod R, so a block never wraps).
//   The scheduler then queues on one HIP stream a staging kernel that reads
//   the pinned staging area over the bus and moves the ranges into the rings
//   (and the cycle's tile queue into device memory), then one persistent
//   launch per base size over a tile queue holding every block pair completed
//   so far on every channel, which writes the outputs straight into a pinned
//   outbox; an event marks the cycle done.  No copy engine takes part, so no
//   dependency between engines has to be resolved by the host.  Up to
//   max_inflight cycles are queued, and chunks that arrive meanwhile go into
//   the next.
//   Completed outputs are moved to per-channel host rings that poll() reads.
//
// Admission: a channel may hold at most R blocks between "received" and
// "polled"; a cycle's staging area and outbox are bounded.  submit() answers
// EXT_EAGAIN when either would overflow; nothing is consumed then.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/qrng_ext.h"
#include "ext_internal.h"
#include "gf2_modulus.h"

using qext::BatchStream;
using qext::BatchTile;
using qext::CombineJob;
using qext::ExtShape;
using qext::ScatterDesc;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Channel {
    bool open = false;
    uint64_t n_bits = 0, nb = 0, qb = 0;
    uint32_t m_bits = 0;
    ExtShape shape{};
    uint32_t slices = 1;          // work-groups per pair (> 1: split into slices)
    uint32_t slice_items = 0;     // items per slice (the last one may hold fewer)
    uint64_t R = 0;               // ring blocks
    uint8_t* ring_x = nullptr;    // device, R * nb bytes
    uint8_t* ring_y = nullptr;
    uint64_t x_recv = 0, y_recv = 0;   // bytes accepted (reserved in some cycle)
    uint64_t x_ok = 0, y_ok = 0;       // bytes scattered by cycles already launched
    uint64_t launched = 0, completed = 0, polled = 0;  // block pairs
    std::vector<uint8_t> out_ring;             // R * qb bytes, slot l mod R
    std::vector<uint64_t> ready_ns;            // R completion times
};

struct Range {
    uint32_t ch;
    uint32_t n;
    uint64_t first_pair;
    uint64_t out_off;     // byte offset in the outbox
    uint64_t part_word0;  // sliced channels: first word of the range's parts
};

// Tiles of one (base size, work-group size, padded) launch while a cycle is built,
// each with its cost (rounds times base products per item).
struct GroupBuild {
    uint32_t bw, threads, padded, lds;
    std::vector<std::pair<uint32_t, BatchTile>> tiles;
};

struct Group {
    uint32_t bw, threads, padded, tile_off, n_tiles, lds_bytes, grid;
};

// A submission's end position on one side, recorded in the cycle that holds it.
struct Resv {
    uint32_t ch;
    uint32_t side;  // 0 = X, 1 = Y
    uint64_t end;
};

struct Slot {
    uint8_t* h_in = nullptr;   // pinned, read by the GPU: data | descs | streams | tiles
    uint8_t* d_in = nullptr;   // device: streams | tiles | queue heads (same offsets)
    uint8_t* h_out = nullptr;  // pinned outbox, written by the GPU
    uint32_t* d_part = nullptr; // device: partial sums of sliced pairs
    hipEvent_t done = nullptr; // the cycle's outputs are in h_out
    hipEvent_t start = nullptr; // before the cycle's first kernel (timing)
    hipEvent_t staged = nullptr;    // after the staging kernel (timing)
    hipEvent_t computed = nullptr;  // after the extraction launches (timing)
    uint64_t data_used = 0;
    uint32_t n_descs = 0;
    int pending = 0;            // submissions still copying into h_in
    std::vector<Resv> resv;
    std::vector<Range> ranges;
    std::vector<Group> groups;
    uint32_t n_tiles = 0;
    uint32_t n_jobs = 0;
    uint32_t combine_lds = 0;
    uint64_t out_bytes = 0;
    uint64_t launched_ns = 0;
    uint64_t table_version = 0;  // server table version last sent to this slot's device copy
};

// Device memory per slot for the partial sums of sliced pairs (a cycle takes
// no more sliced pairs than fit; the rest wait for the next cycle).
constexpr uint64_t kPartBytes = 32ull << 20;

}  // namespace

struct ext_server {
    int device = 0;
    hipStream_t stream = nullptr;        // extraction and combine launches
    hipStream_t stage_stream = nullptr;  // staging kernels (library-owned)
    bool own_stream = false;
    int cus = 1;
    uint32_t lds_per_cu = 65536;     // LDS bytes per CU
    uint32_t lds_per_block = 65536;  // largest LDS request of one work-group
    ext_server_config cfg{};
    ext_params params{};
    std::vector<Channel> ch;
    // slot layout
    size_t off_desc = 0, off_streams = 0, off_tiles = 0, off_heads = 0, in_bytes = 0;
    uint32_t max_jobs = 0;  // combine jobs per cycle (each has at least two tiles)
    static constexpr int kSlots = 4;  // one filling, up to kMaxInflight in flight
    static constexpr uint32_t kMaxInflight = kSlots - 1;
    Slot slots[kSlots];
    int filling = 0;
    bool launching = false;  // a slot has been taken and its kernels are not all queued yet
    std::deque<int> inflight;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, int> occ_cache;  // (bw, threads, lds)
    std::mutex mu;
    std::condition_variable cv;
    std::condition_variable ready_cv;  // signalled when a cycle's outputs land
    int ready_waiters = 0;
    std::thread sched;
    bool stop = false;
    int sticky = EXT_OK;
    ext_server_stats stats{};
    std::vector<CombineJob> jobs_tmp;  // launch_cycle's job list (kept to reuse its storage)
    std::vector<GroupBuild> group_build;  // launch_cycle's tile lists (likewise)
    uint64_t table_version = 1;        // bumped whenever a channel opens or closes
};

namespace {

void server_free(ext_server* s) {
    for (Slot& sl : s->slots) {
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        (void)hipFree(sl.d_in);
        (void)hipFree(sl.d_part);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.start) (void)hipEventDestroy(sl.start);
        if (sl.staged) (void)hipEventDestroy(sl.staged);
        if (sl.computed) (void)hipEventDestroy(sl.computed);
    }
    for (Channel& c : s->ch) {
        (void)hipFree(c.ring_x);
        (void)hipFree(c.ring_y);
    }
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->stage_stream) (void)hipStreamDestroy(s->stage_stream);
    delete s;
}

// Move finished cycles' outputs into the channels' host rings (lock held).
void harvest(ext_server* s) {
    while (!s->inflight.empty()) {
        Slot& sl = s->slots[s->inflight.front()];
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) return;
        if (q != hipSuccess) {
            s->sticky = EXT_EDEVICE;
            return;
        }
        const uint64_t t = now_ns();
        for (const Range& r : sl.ranges) {
            Channel& c = s->ch[r.ch];
            for (uint32_t k = 0; k < r.n; ++k) {
                const uint64_t slot = (r.first_pair + k) % c.R;
                memcpy(c.out_ring.data() + slot * c.qb, sl.h_out + r.out_off + k * c.qb, c.qb);
                c.ready_ns[slot] = t;
            }
            c.completed += r.n;
        }
        s->stats.gpu_busy_ns += t - sl.launched_ns;
        if (s->cfg.timing) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, sl.start, sl.done) == hipSuccess)
                s->stats.gpu_ns += (uint64_t)(ms * 1e6f);
            if (hipEventElapsedTime(&ms, sl.start, sl.staged) == hipSuccess)
                s->stats.stage_ns += (uint64_t)(ms * 1e6f);
            if (hipEventElapsedTime(&ms, sl.staged, sl.computed) == hipSuccess)
                s->stats.extract_ns += (uint64_t)(ms * 1e6f);
        }
        s->stats.max_cycle_ns = std::max(s->stats.max_cycle_ns, t - sl.launched_ns);
        if (s->ready_waiters && !sl.ranges.empty()) s->ready_cv.notify_all();
        sl.ranges.clear();
        sl.data_used = 0;
        sl.n_descs = 0;
        s->inflight.pop_front();
    }
}

int occupancy(ext_server* s, uint32_t bw, uint32_t threads, uint32_t padded, uint32_t lds) {
    auto key = std::make_tuple(bw, threads * 2 + padded, lds);
    auto it = s->occ_cache.find(key);
    if (it != s->occ_cache.end()) return it->second;
    int occ = 0;
    if (qext::batch_occupancy(bw, threads, padded != 0, lds, &occ) != hipSuccess || occ <= 0)
        occ = 1;
    s->occ_cache[key] = occ;
    return occ;
}

// Take the filling slot, add every ready block pair, and queue the cycle
// (lock held on entry and exit; released around the HIP calls).
int launch_cycle(ext_server* s, std::unique_lock<std::mutex>& lk) {
    const uint64_t t_enter = now_ns();
    // While set, ext_server_close waits: the taken slot may hold scatter
    // descriptors into a closing channel's rings, and its staging kernel is
    // queued without the lock.  Cleared (lock held) on every return.
    struct Launching {
        ext_server* s;
        ~Launching() {
            s->launching = false;
            s->cv.notify_all();
        }
    } launching_guard{s};
    s->launching = true;
    const int idx = s->filling;
    Slot& sl = s->slots[idx];
    // the next filling slot: one that is neither in flight nor this one
    int next = -1;
    for (int k = 0; k < ext_server::kSlots; ++k) {
        if (k == idx) continue;
        if (std::find(s->inflight.begin(), s->inflight.end(), k) == s->inflight.end()) next = k;
    }
    if (next < 0) return EXT_OK;
    // new submissions go to `next` from here on; wait for copies into this one
    s->filling = next;
    while (sl.pending > 0) s->cv.wait(lk);
    for (const Resv& r : sl.resv) {
        Channel& c = s->ch[r.ch];
        uint64_t& ok = r.side ? c.y_ok : c.x_ok;
        ok = std::max(ok, r.end);
    }
    sl.resv.clear();

    // Under the lock: every channel's ready pairs as ranges (at most one per
    // ring pass), within the cycle's outbox, tile, job and part limits.  A
    // sliced pair takes `slices` tiles, room for their parts and one combine
    // job; other pairs go ppw to a tile.
    uint64_t out_off = 0, part_words = 0;
    const uint64_t part_cap = kPartBytes / 4;
    uint32_t n_tiles = 0, n_jobs = 0;
    sl.ranges.clear();
    for (uint32_t ci = 0; ci < s->ch.size(); ++ci) {
        Channel& c = s->ch[ci];
        if (!c.open) continue;
        uint64_t ready = std::min(c.x_ok, c.y_ok) / c.nb - c.launched;
        const uint64_t cw = 2ull * c.shape.qw;
        while (ready) {
            const uint64_t slot0 = c.launched % c.R;
            out_off = align_up(out_off, 4);  // word stores for 32-bit multiple degrees
            uint64_t k = std::min<uint64_t>(ready, c.R - slot0);            // no ring wrap
            k = std::min<uint64_t>(k, out_off < s->cfg.outbox_bytes
                                          ? (s->cfg.outbox_bytes - out_off) / c.qb
                                          : 0);  // outbox room
            uint64_t part0 = 0;
            if (c.slices > 1) {
                k = std::min<uint64_t>(k, (s->cfg.max_tiles - n_tiles) / c.slices);
                k = std::min<uint64_t>(k, s->max_jobs - n_jobs);
                part0 = align_up(part_words, 4);  // 16-byte aligned parts
                k = std::min<uint64_t>(k, part0 < part_cap ? (part_cap - part0) / (c.slices * cw) : 0);
            } else {
                const uint64_t tiles_needed = (k + c.shape.ppw - 1) / c.shape.ppw;
                if (n_tiles + tiles_needed > s->cfg.max_tiles)
                    k = std::min<uint64_t>(k, (uint64_t)(s->cfg.max_tiles - n_tiles) * c.shape.ppw);
            }
            if (k == 0) break;
            sl.ranges.push_back(Range{ci, (uint32_t)k, c.launched, out_off, part0});
            if (c.slices > 1) {
                n_tiles += (uint32_t)k * c.slices;
                n_jobs += (uint32_t)k;
                part_words = part0 + k * c.slices * cw;
                s->stats.split_pairs += k;
            } else {
                n_tiles += (uint32_t)((k + c.shape.ppw - 1) / c.shape.ppw);
            }
            out_off += k * c.qb;
            c.launched += k;
            ready -= k;
        }
    }
    if (sl.data_used == 0 && n_tiles == 0) return EXT_OK;  // (the slot stays free)

    // the stream table only when a channel opened or closed since this slot
    // last sent it (written under the lock: open() changes the channels)
    const bool send_table = sl.table_version != s->table_version;
    if (send_table) {
        BatchStream* hs = reinterpret_cast<BatchStream*>(sl.h_in + s->off_streams);
        for (uint32_t ci = 0; ci < s->ch.size(); ++ci) {
            const Channel& c = s->ch[ci];
            hs[ci] = BatchStream{c.ring_x, c.ring_y, sl.h_out, 0, c.shape};
        }
        sl.table_version = s->table_version;
    }
    s->inflight.push_back(idx);
    s->stats.cycles += 1;
    s->stats.tiles += n_tiles;
    for (const Range& r : sl.ranges) s->stats.pairs += r.n;

    // Without the lock (submit() fills `next`, poll() reads harvested cycles;
    // the channels of these ranges stay open until their pairs complete):
    // tiles grouped by (base size, work-group size), longest first, since a
    // lane's critical path is its rounds times the base products per item.
    lk.unlock();
    std::vector<GroupBuild>& gb = s->group_build;
    for (GroupBuild& g : gb) g.tiles.clear();
    std::vector<CombineJob>& jobs = s->jobs_tmp;
    jobs.clear();
    uint32_t combine_lds = 0;
    for (const Range& r : sl.ranges) {
        const Channel& c = s->ch[r.ch];
        const ExtShape& sh = c.shape;
        GroupBuild* g = nullptr;
        for (GroupBuild& x : gb)
            if (x.bw == sh.bw && x.threads == sh.threads && x.padded == sh.padded) g = &x;
        if (!g) {
            gb.push_back(GroupBuild{sh.bw, sh.threads, sh.padded, 0, {}});
            g = &gb.back();
        }
        if (g->tiles.empty()) g->lds = 0;
        g->lds = std::max(g->lds, qext::group_lds_bytes(sh));
        const uint64_t slot0 = r.first_pair % c.R;
        if (c.slices > 1) {
            const uint32_t items = sh.np * sh.n_e;
            const uint64_t cw = 2ull * sh.qw;
            uint64_t pw = r.part_word0;
            for (uint64_t p = 0; p < r.n; ++p) {
                jobs.push_back(CombineJob{r.ch, c.slices, pw, r.out_off + p * c.qb});
                for (uint32_t sidx = 0; sidx < c.slices; ++sidx) {
                    const uint32_t i0 = sidx * c.slice_items;
                    const uint32_t ni = std::min(c.slice_items, items - i0);
                    g->tiles.push_back({(ni + sh.threads - 1) / sh.threads,
                                        BatchTile{r.ch, 1, slot0 + p, pw, i0, ni}});
                    pw += cw;
                }
            }
            combine_lds = std::max<uint32_t>(combine_lds, (uint32_t)(cw + sh.dn) * 4);
        } else {
            for (uint64_t p = 0; p < r.n; p += sh.ppw) {
                const uint32_t n = (uint32_t)std::min<uint64_t>(sh.ppw, r.n - p);
                const uint64_t items = (uint64_t)n * sh.np * sh.groups;
                const uint32_t cost = (uint32_t)(((items + sh.threads - 1) / sh.threads) * sh.epg);
                g->tiles.push_back(
                    {cost, BatchTile{r.ch, n, slot0 + p, r.out_off + p * c.qb, 0, 0}});
            }
        }
    }
    BatchTile* ht = reinterpret_cast<BatchTile*>(sl.h_in + s->off_tiles);
    sl.groups.clear();
    uint32_t t_off = 0;
    for (GroupBuild& gr : gb) {
        if (gr.tiles.empty()) continue;
        std::stable_sort(gr.tiles.begin(), gr.tiles.end(),
                         [](const std::pair<uint32_t, BatchTile>& a,
                            const std::pair<uint32_t, BatchTile>& b) { return a.first > b.first; });
        Group g{gr.bw, gr.threads, gr.padded, t_off, (uint32_t)gr.tiles.size(), gr.lds, 0};
        for (size_t i = 0; i < gr.tiles.size(); ++i) ht[t_off + i] = gr.tiles[i].second;
        int per_cu = occupancy(s, g.bw, g.threads, g.padded, g.lds_bytes);
        if (s->cfg.wg_per_cu && (int)s->cfg.wg_per_cu < per_cu) {
            // at most wg_per_cu groups per CU: ask for just over 1/(k+1) of the
            // CU's LDS, so the dispatcher cannot stack more groups on one CU
            // (long tiles then keep their SIMDs to themselves)
            const uint32_t k = s->cfg.wg_per_cu;
            const uint32_t pad = s->lds_per_cu / (k + 1) + 256;
            if (pad <= s->lds_per_block) {
                g.lds_bytes = std::max(g.lds_bytes, pad);
                per_cu = (int)k;
            }
        }
        g.grid = (uint32_t)std::min<uint64_t>(g.n_tiles, (uint64_t)s->cus * per_cu);
        t_off += g.n_tiles;
        sl.groups.push_back(g);
    }
    // combine jobs right after the used tiles (one metadata copy covers both)
    const size_t off_jobs = align_up(s->off_tiles + (size_t)n_tiles * sizeof(BatchTile), 16);
    if (!jobs.empty())
        memcpy(sl.h_in + off_jobs, jobs.data(), jobs.size() * sizeof(CombineJob));
    sl.n_tiles = n_tiles;
    sl.n_jobs = (uint32_t)jobs.size();
    sl.combine_lds = combine_lds;
    sl.out_bytes = out_off;

    hipError_t e = hipSuccess;
    // staging (reads the pinned area over the bus), then one persistent launch
    // per base size writing outputs straight into the pinned outbox, then the
    // combine step of sliced pairs
    const size_t meta_off = send_table ? s->off_streams : s->off_tiles;
    const size_t meta_bytes =
        (off_jobs + (size_t)sl.n_jobs * sizeof(CombineJob) - meta_off + 15) / 16 * 16;
    sl.launched_ns = now_ns();
    const uint64_t t_built = sl.launched_ns;
    // staging on its own stream, so that it overlaps the previous cycle's
    // extraction; the compute stream waits for it on the GPU
    if (s->cfg.timing) e = hipEventRecord(sl.start, s->stage_stream);
    if (e == hipSuccess)
        e = qext::launch_stage(sl.h_in, reinterpret_cast<const ScatterDesc*>(sl.h_in + s->off_desc),
                           sl.n_descs, sl.h_in + meta_off, sl.d_in + meta_off,
                           (uint32_t)meta_bytes, reinterpret_cast<uint32_t*>(sl.d_in + s->off_heads),
                           (uint32_t)sl.groups.size(), s->stage_stream);
    if (e == hipSuccess) e = hipEventRecord(sl.staged, s->stage_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, sl.staged, 0);
    for (size_t gi = 0; gi < sl.groups.size() && e == hipSuccess; ++gi) {
        const Group& g = sl.groups[gi];
        e = qext::launch_batch_noreset(
            g.bw, g.threads, g.padded != 0,
            reinterpret_cast<const BatchStream*>(sl.d_in + s->off_streams),
            reinterpret_cast<const BatchTile*>(sl.d_in + s->off_tiles) + g.tile_off, g.n_tiles,
            reinterpret_cast<uint32_t*>(sl.d_in + s->off_heads) + gi, sl.d_part, g.grid,
            g.lds_bytes, s->stream);
    }
    if (e == hipSuccess && s->cfg.timing) e = hipEventRecord(sl.computed, s->stream);
    if (e == hipSuccess && sl.n_jobs)
        e = qext::launch_combine(
            reinterpret_cast<const BatchStream*>(sl.d_in + s->off_streams),
            reinterpret_cast<const CombineJob*>(sl.d_in + off_jobs), sl.n_jobs, sl.d_part,
            (uint32_t)std::min<uint64_t>(sl.n_jobs, (uint64_t)s->cus * 4), sl.combine_lds,
            s->stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, s->stream);
    const uint64_t t_queued = now_ns();
    lk.lock();
    s->stats.build_ns += t_built - t_enter;
    s->stats.launch_ns += t_queued - t_built;
    if (e != hipSuccess) {
        s->sticky = EXT_EDEVICE;
        return EXT_EDEVICE;
    }
    return EXT_OK;
}

// A new cycle may start once the newest cycle in flight has been staged (its
// staging kernel then no longer holds the staging stream).
bool stage_free(ext_server* s) {
    if (s->inflight.empty()) return true;
    return hipEventQuery(s->slots[s->inflight.back()].staged) == hipSuccess;
}

bool has_work(ext_server* s) {
    if (s->slots[s->filling].data_used) return true;
    for (const Channel& c : s->ch)
        if (c.open && std::min(c.x_ok, c.y_ok) / c.nb > c.launched) return true;
    return false;
}

void scheduler(ext_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop && s->inflight.empty()) break;
        harvest(s);
        if (s->sticky) {
            s->cv.notify_all();
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
            if (s->stop) break;
            continue;
        }
        if (!s->stop && s->inflight.size() < (size_t)s->cfg.max_inflight && has_work(s) &&
            stage_free(s)) {
            launch_cycle(s, lk);
            s->cv.notify_all();
            continue;
        }
        if (!s->inflight.empty()) {
            // a cycle is on the GPU: look again at once (a timed wait sleeps for
            // tens of microseconds at least), or after poll_us if configured
            if (s->cfg.poll_us > 1) {
                s->cv.wait_for(lk, std::chrono::microseconds(s->cfg.poll_us));
            } else {
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            }
        } else {
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }
}

}  // namespace

extern "C" {

void ext_server_config_init(ext_server_config* c) {
    if (!c) return;
    memset(c, 0, sizeof *c);
    c->max_channels = 256;
    c->ring_blocks = 0;
    c->ring_bytes = 4ull << 20;
    c->stage_bytes = 64ull << 20;
    c->outbox_bytes = 32ull << 20;
    c->max_tiles = 1u << 17;
    c->max_inflight = 2;
    c->split_pairs = 1;
    c->max_descs = 1u << 16;
    c->poll_us = 0;
    c->device_reserve_bytes = 1ull << 30;
    c->rings_bytes_cap = 0;
}

int ext_server_create(const ext_server_config* cfg, const ext_params* p, ext_server** out) {
    if (!out) return EXT_EINVAL;
    *out = nullptr;
    ext_server_config dc;
    ext_server_config_init(&dc);
    if (!cfg) cfg = &dc;
    ext_params dp;
    ext_params_init(&dp);
    if (!p) p = &dp;
    if (p->n_taps || cfg->max_channels == 0 || (cfg->ring_blocks == 0 && cfg->ring_bytes == 0) ||
        cfg->stage_bytes == 0 ||
        cfg->outbox_bytes < 4 || cfg->max_tiles == 0 || cfg->max_descs < 4 ||
        cfg->max_inflight == 0 || cfg->max_inflight > ext_server::kMaxInflight ||
        p->kernel > EXT_KERNEL_BITSLICE)
        return EXT_EINVAL;
    if (p->kernel == EXT_KERNEL_BITSLICE) return EXT_ENOTSUP;  // word-level kernels only
    ext_server* s = new (std::nothrow) ext_server;
    if (!s) return EXT_ENOMEM;
    s->cfg = *cfg;
    s->params = *p;
    int dev = p->device;
    if ((dev < 0 && hipGetDevice(&dev) != hipSuccess) || hipSetDevice(dev) != hipSuccess) {
        delete s;
        return EXT_EDEVICE;
    }
    s->device = dev;
    if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        s->cus = 1;
    {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
                hipSuccess && v > 0)
            s->lds_per_cu = (uint32_t)v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            s->lds_per_block = (uint32_t)v;
    }
    if (p->use_hip_stream && p->hip_stream) {
        s->stream = (hipStream_t)p->hip_stream;
    } else if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess) {
        s->own_stream = true;
    } else {
        delete s;
        return EXT_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&s->stage_stream, hipStreamNonBlocking) != hipSuccess) {
        s->stage_stream = nullptr;
        server_free(s);
        return EXT_EDEVICE;
    }
    s->off_desc = align_up(cfg->stage_bytes, 256);
    s->off_streams = align_up(s->off_desc + (size_t)cfg->max_descs * sizeof(ScatterDesc), 256);
    s->off_tiles = align_up(s->off_streams + (size_t)cfg->max_channels * sizeof(BatchStream), 256);
    s->max_jobs = cfg->max_tiles / 2;
    // tiles, then (16-byte aligned) combine jobs; +16: the metadata copy is
    // rounded up to 16 bytes
    s->off_heads = align_up(s->off_tiles + (size_t)cfg->max_tiles * sizeof(BatchTile) + 16 +
                                (size_t)s->max_jobs * sizeof(CombineJob) + 16,
                            256);
    s->in_bytes = s->off_heads + 64 * sizeof(uint32_t);
    bool ok = true;
    for (Slot& sl : s->slots) {
        // coherent (fine-grained) host memory: the GPU reads the staging area
        // and writes the outbox over the bus, visible once the cycle's event is
        ok = ok && hipHostMalloc((void**)&sl.h_in, s->in_bytes, hipHostMallocCoherent) == hipSuccess;
        ok = ok && hipHostMalloc((void**)&sl.h_out, cfg->outbox_bytes, hipHostMallocCoherent) ==
                       hipSuccess;
        ok = ok && hipMalloc((void**)&sl.d_in, s->in_bytes) == hipSuccess;
        ok = ok && hipMalloc((void**)&sl.d_part, kPartBytes) == hipSuccess;
        const unsigned ev_flags = cfg->timing ? hipEventDefault : hipEventDisableTiming;
        ok = ok && hipEventCreateWithFlags(&sl.done, ev_flags) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.staged, ev_flags) == hipSuccess;
        if (cfg->timing) {
            ok = ok && hipEventCreate(&sl.start) == hipSuccess;
            ok = ok && hipEventCreate(&sl.computed) == hipSuccess;
        }
    }
    try {
        s->ch.resize(cfg->max_channels);
    } catch (const std::bad_alloc&) {
        ok = false;
    }
    if (!ok) {
        (void)hipGetLastError();
        server_free(s);
        return EXT_ENOMEM;
    }
    try {
        s->sched = std::thread(scheduler, s);
    } catch (...) {
        server_free(s);
        return EXT_ENOMEM;
    }
    *out = s;
    return EXT_OK;
}

int ext_server_open(ext_server* s, uint64_t n_bits, uint32_t m_bits, uint32_t* channel) {
    if (!s || !channel || n_bits == 0 || m_bits == 0 || n_bits % m_bits ||
        n_bits / m_bits > 0xffffffffull)
        return EXT_EINVAL;
    std::vector<uint32_t> taps;
    try {
        if (!qext::default_modulus(m_bits, &taps)) return EXT_ENOTSUP;
    } catch (const std::bad_alloc&) {
        return EXT_ENOMEM;
    }
    const uint32_t n_e = (uint32_t)(n_bits / m_bits);
    qext::PlanKnobs knobs{s->params.base_bits / 32, s->params.groups, s->params.pairs_per_group,
                          s->params.threads};
    // latency plan: one base product per item (every element its own group),
    // so no lane runs a chain of n_e products
    if (s->cfg.split_pairs && !knobs.groups && !s->params.autotune) knobs.groups = n_e;
    if (s->params.autotune &&
        qext::autotune_shape(m_bits, n_e, taps.data(), (uint32_t)taps.size(), s->stream, &knobs,
                             nullptr) != hipSuccess)
        return EXT_EDEVICE;
    ExtShape shape;
    if (!qext::plan_shape(m_bits, n_e, taps.data(), (uint32_t)taps.size(), knobs, &shape))
        return EXT_ENOTSUP;
    const uint64_t nb = n_bits / 8, qb = m_bits / 8;
    if (qb > s->cfg.outbox_bytes) return EXT_EINVAL;
    // pairs with more (element, sub-product) items than lanes: split over
    // ceil(items / threads) work-groups
    uint32_t slices = 1, slice_items = 0;
    {
        const uint64_t items = (uint64_t)shape.np * n_e;
        if (s->cfg.split_pairs && items > shape.threads && !shape.padded) {
            // per <= threads items per slice; every slice but the last holds
            // exactly per, the last at least one
            const uint64_t per = (items + (items + shape.threads - 1) / shape.threads - 1) /
                                 ((items + shape.threads - 1) / shape.threads);
            const uint64_t sl = (items + per - 1) / per;
            if (items > 0xffffffffull || sl * 2ull * shape.qw * 4 > kPartBytes ||
                sl > s->cfg.max_tiles / 2 || (2ull * shape.qw + shape.dn) * 4 > 65536)
                return EXT_ENOTSUP;
            slices = (uint32_t)sl;
            slice_items = (uint32_t)per;
        }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->sticky) return s->sticky;
    uint32_t ci = 0;
    while (ci < s->ch.size() && (s->ch[ci].open || s->ch[ci].ring_x)) ++ci;
    if (ci == s->ch.size()) return EXT_EAGAIN;
    Channel& c = s->ch[ci];
    c = Channel{};
    c.n_bits = n_bits;
    c.m_bits = m_bits;
    c.nb = nb;
    c.qb = qb;
    c.shape = shape;
    c.slices = slices;
    c.slice_items = slice_items;
    c.R = s->cfg.ring_blocks ? s->cfg.ring_blocks
                             : std::max<uint64_t>(128, s->cfg.ring_bytes / nb);
    // admission by free device memory: the two rings must fit in what the
    // device has free less the reserve, and under the cap on all rings
    const uint64_t need = 2 * c.R * nb;
    if (hipSetDevice(s->device) != hipSuccess) {
        (void)hipGetLastError();
        c = Channel{};
        return EXT_EDEVICE;
    }
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            c = Channel{};
            return EXT_EDEVICE;
        }
        s->stats.free_bytes = free_b;
        const bool over_free = (uint64_t)free_b < s->cfg.device_reserve_bytes ||
                               need > (uint64_t)free_b - s->cfg.device_reserve_bytes;
        const bool over_cap = s->cfg.rings_bytes_cap &&
                              s->stats.rings_bytes + need > s->cfg.rings_bytes_cap;
        if (over_free || over_cap) {
            s->stats.eagain_mem += 1;
            c = Channel{};
            return EXT_EAGAIN;
        }
    }
    try {
        c.out_ring.resize(c.R * qb);
        c.ready_ns.resize(c.R);
    } catch (const std::bad_alloc&) {
        return EXT_ENOMEM;
    }
    if (hipMalloc((void**)&c.ring_x, c.R * nb) != hipSuccess ||
        hipMalloc((void**)&c.ring_y, c.R * nb) != hipSuccess) {
        (void)hipFree(c.ring_x);
        (void)hipFree(c.ring_y);
        c.ring_x = c.ring_y = nullptr;
        (void)hipGetLastError();
        return EXT_ENOMEM;
    }
    c.open = true;
    s->stats.rings_bytes += need;
    s->table_version += 1;
    *channel = ci;
    return EXT_OK;
}

int ext_server_submit(ext_server* s, uint32_t channel, const void* x, size_t x_len, const void* y,
                      size_t y_len) {
    if (!s || (x_len && !x) || (y_len && !y)) return EXT_EINVAL;
    if (x_len > 0xffffffffull || y_len > 0xffffffffull) return EXT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->sticky) return s->sticky;
    if (channel >= s->ch.size() || !s->ch[channel].open) return EXT_ECLOSED;
    Channel& c = s->ch[channel];
    const uint64_t limit = (c.polled + c.R) * c.nb;
    if (c.x_recv + x_len > limit || c.y_recv + y_len > limit) {
        s->stats.eagain_ring += 1;
        return EXT_EAGAIN;
    }
    Slot& sl = s->slots[s->filling];
    // descriptors: one per 16 KiB piece, plus one per side for the ring wrap
    const uint64_t need_descs = (x_len + 16383) / 16384 + (y_len + 16383) / 16384 + 4;
    if (sl.data_used + x_len + y_len > s->cfg.stage_bytes ||
        sl.n_descs + need_descs > s->cfg.max_descs) {
        s->stats.eagain_stage += 1;
        s->cv.notify_all();
        return EXT_EAGAIN;
    }
    // reserve staging space and descriptors, then copy without the lock
    const uint64_t ring_bytes = c.R * c.nb;
    ScatterDesc* descs = reinterpret_cast<ScatterDesc*>(sl.h_in + s->off_desc);
    uint8_t* dst_x = sl.h_in + sl.data_used;
    // copy ranges of at most kPiece bytes, none crossing the ring's end, so the
    // scatter kernel spreads a large chunk over many work-groups
    constexpr uint64_t kPiece = 16384;
    auto reserve = [&](size_t len, uint64_t pos, uint8_t* ring) {
        uint64_t done = 0;
        while (done < len) {
            const uint64_t off = (pos + done) % ring_bytes;
            const uint64_t k = std::min<uint64_t>({len - done, ring_bytes - off, kPiece});
            descs[sl.n_descs++] = ScatterDesc{sl.data_used + done, ring + off, (uint32_t)k, channel};
            done += k;
        }
        sl.data_used += len;
    };
    if (x_len) {
        reserve(x_len, c.x_recv, c.ring_x);
        c.x_recv += x_len;
        sl.resv.push_back(Resv{channel, 0, c.x_recv});
    }
    uint8_t* dst_y = sl.h_in + sl.data_used;
    if (y_len) {
        reserve(y_len, c.y_recv, c.ring_y);
        c.y_recv += y_len;
        sl.resv.push_back(Resv{channel, 1, c.y_recv});
    }
    sl.pending += 1;
    s->stats.bytes_in += x_len + y_len;
    lk.unlock();
    if (x_len) memcpy(dst_x, x, x_len);
    if (y_len) memcpy(dst_y, y, y_len);
    lk.lock();
    sl.pending -= 1;
    s->cv.notify_all();
    return EXT_OK;
}

int ext_server_poll(ext_server* s, uint32_t channel, void* out, size_t out_cap, size_t* out_len,
                    uint64_t* ready_ns, uint64_t* blocks_done) {
    if (!s || (out_cap && !out)) return EXT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->sticky) return s->sticky;
    if (channel >= s->ch.size() || !s->ch[channel].open) return EXT_ECLOSED;
    Channel& c = s->ch[channel];
    const uint64_t k = std::min<uint64_t>(c.completed - c.polled, out_cap / c.qb);
    for (uint64_t i = 0; i < k; ++i) {
        const uint64_t slot = (c.polled + i) % c.R;
        memcpy((uint8_t*)out + i * c.qb, c.out_ring.data() + slot * c.qb, c.qb);
        if (ready_ns) ready_ns[i] = c.ready_ns[slot];
    }
    c.polled += k;
    if (out_len) *out_len = k * c.qb;
    if (blocks_done) *blocks_done = c.polled;
    if (k) s->cv.notify_all();
    return EXT_OK;
}

int ext_server_ready(ext_server* s, uint32_t* chans, uint32_t cap, uint32_t* n,
                     uint32_t timeout_us) {
    if (!s || !n || (cap && !chans)) return EXT_EINVAL;
    *n = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    auto collect = [&] {
        uint32_t k = 0;
        for (uint32_t ci = 0; ci < s->ch.size() && k < cap; ++ci) {
            const Channel& c = s->ch[ci];
            if (c.open && c.completed > c.polled) chans[k++] = ci;
        }
        return k;
    };
    uint32_t k = collect();
    if (!k && timeout_us) {
        s->ready_waiters += 1;
        s->ready_cv.wait_for(lk, std::chrono::microseconds(timeout_us));
        s->ready_waiters -= 1;
        k = collect();
    }
    *n = k;
    return s->sticky;
}

int ext_server_close(ext_server* s, uint32_t channel, uint64_t* dropped_bits) {
    if (!s) return EXT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (channel >= s->ch.size() || !s->ch[channel].open) return EXT_ECLOSED;
    Channel& c = s->ch[channel];
    // let every launched pair of this channel finish before its rings go
    while (c.completed < c.launched && !s->sticky) {
        s->cv.notify_all();
        s->cv.wait_for(lk, std::chrono::microseconds(200));
    }
    const uint64_t full = std::min(c.x_recv, c.y_recv) / c.nb;
    if (dropped_bits) *dropped_bits = 8 * (std::max(c.x_recv, c.y_recv) - full * c.nb);
    c.open = false;
    s->table_version += 1;
    // bytes of this channel still waiting in the filling cycle must not be
    // scattered into rings that are about to be freed
    {
        Slot& sl = s->slots[s->filling];
        while (sl.pending > 0) s->cv.wait(lk);
        ScatterDesc* descs = reinterpret_cast<ScatterDesc*>(sl.h_in + s->off_desc);
        for (uint32_t i = 0; i < sl.n_descs; ++i)
            if (descs[i].pad == channel) descs[i].len = 0;
        sl.resv.erase(std::remove_if(sl.resv.begin(), sl.resv.end(),
                                     [&](const Resv& r) { return r.ch == channel; }),
                      sl.resv.end());
    }
    // a cycle being built may hold this channel's bytes in the slot it took
    // before the close: once its kernels are queued, the stream syncs below
    // cover its staging
    while (s->launching) s->cv.wait(lk);
    // pairs received but not yet launched are dropped with the channel; wait
    // for the stream before freeing the rings
    lk.unlock();
    (void)hipStreamSynchronize(s->stage_stream);
    (void)hipStreamSynchronize(s->stream);
    lk.lock();
    (void)hipFree(c.ring_x);
    (void)hipFree(c.ring_y);
    c.ring_x = c.ring_y = nullptr;
    s->stats.rings_bytes -= 2 * c.R * c.nb;
    return EXT_OK;
}

int ext_server_stats_get(ext_server* s, ext_server_stats* out) {
    if (!s || !out) return EXT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    *out = s->stats;
    return s->sticky;
}

int ext_server_destroy(ext_server* s) {
    if (!s) return EXT_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
        s->ready_cv.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    (void)hipStreamSynchronize(s->stream);
    server_free(s);
    return EXT_OK;
}

}  // extern "C"
