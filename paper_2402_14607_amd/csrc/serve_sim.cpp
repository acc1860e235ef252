// serve_sim.cpp -- real-time load generator for the served form.
//
// Channel c receives chunks at the jumps of a Poisson process of rate
// lambda_c = (raw_bytes_per_s / n_channels) / (2 * nb_c * mean_k); a chunk is
// k blocks of X and k blocks of Y (k uniform on [min, max]), read cyclically
// from the channel's pools.  Producer threads (channels split among them)
// submit every chunk at its scheduled time (or as soon after as admission
// allows); a consumer thread
// polls every channel and takes, for each returned block, the latency from
// the scheduled arrival of the chunk that completed it to the poll that
// returned it.  The same trace can drive the server or the plain streaming
// form (one ext_stream, hence one launch per chunk, per channel).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <thread>
#include <vector>

#include "../../include/qrng_ext.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Event {
    uint64_t t_ns;  // scheduled arrival, relative to the start
    uint32_t ch;
    uint32_t k;     // blocks per side
};

struct Chan {
    std::mutex mu;  // guards the bookkeeping below and, in plain mode, the ext_stream
    uint64_t nb = 0, qb = 0;
    struct Rec {
        uint64_t end;        // blocks submitted after this chunk
        uint64_t arrival;    // scheduled arrival, ns
        uint64_t submitted;  // when its submission returned, ns
    };
    std::deque<Rec> chunks;
    uint64_t submitted = 0;  // blocks submitted (per side)
    uint64_t returned = 0;   // blocks returned by polls
    uint64_t pool_pos = 0;
    uint64_t captured = 0;
    uint32_t sid = 0;                // served mode channel index
    ext_ctx* ctx = nullptr;          // plain mode
    ext_stream* st = nullptr;
};

}  // namespace

extern "C" int ext_serve_simulate(const ext_sim_config* cfg, ext_sim_result* res,
                                  uint64_t* capture_len) {
    if (!cfg || !res || cfg->n_channels == 0 || !cfg->n_bits || !cfg->m_bits || !cfg->pool_x ||
        !cfg->pool_y || !cfg->pool_bytes || cfg->raw_bytes_per_s <= 0 ||
        cfg->min_chunk_blocks == 0 || cfg->max_chunk_blocks < cfg->min_chunk_blocks ||
        cfg->duration_s <= 0 || cfg->warmup_s < 0 || cfg->grace_s < 0 ||
        (cfg->mode != EXT_SIM_SERVED && cfg->mode != EXT_SIM_PLAIN))
        return EXT_EINVAL;
    memset(res, 0, sizeof *res);
    const uint32_t nc = cfg->n_channels;
    std::vector<std::unique_ptr<Chan>> ch;
    for (uint32_t c = 0; c < nc; ++c) {
        ch.emplace_back(new Chan);
        ch[c]->nb = cfg->n_bits[c] / 8;
        ch[c]->qb = cfg->m_bits[c] / 8;
        if (!ch[c]->nb || !ch[c]->qb || cfg->pool_bytes[c] < cfg->max_chunk_blocks * ch[c]->nb ||
            cfg->pool_bytes[c] % ch[c]->nb)
            return EXT_EINVAL;
    }

    // ---- schedule ---------------------------------------------------------
    const double horizon = cfg->warmup_s + cfg->duration_s;
    std::vector<Event> ev;
    std::mt19937_64 rng(cfg->seed);
    const double mean_k = 0.5 * (cfg->min_chunk_blocks + cfg->max_chunk_blocks);
    double offered_bits = 0;
    for (uint32_t c = 0; c < nc; ++c) {
        const double lam = cfg->raw_bytes_per_s / nc / (2.0 * ch[c]->nb * mean_k);
        std::exponential_distribution<double> gap(lam);
        std::uniform_int_distribution<uint32_t> kdist(cfg->min_chunk_blocks, cfg->max_chunk_blocks);
        double t = gap(rng);
        while (t < horizon) {
            const uint32_t k = kdist(rng);
            ev.push_back(Event{(uint64_t)(t * 1e9), c, k});
            if (t >= cfg->warmup_s) offered_bits += 16.0 * k * ch[c]->nb;
            t += gap(rng);
        }
    }
    std::sort(ev.begin(), ev.end(), [](const Event& a, const Event& b) { return a.t_ns < b.t_ns; });

    // ---- set up the system under test --------------------------------------
    ext_server* srv = nullptr;
    int rc = EXT_OK;
    if (cfg->mode == EXT_SIM_SERVED) {
        rc = ext_server_create(cfg->server_cfg, cfg->params, &srv);
        for (uint32_t c = 0; c < nc && rc == EXT_OK; ++c)
            rc = ext_server_open(srv, cfg->n_bits[c], cfg->m_bits[c], &ch[c]->sid);
    } else {
        ext_params p;
        if (cfg->params)
            p = *cfg->params;
        else
            ext_params_init(&p);
        p.mem_kind = EXT_MEM_HOST;
        for (uint32_t c = 0; c < nc && rc == EXT_OK; ++c) {
            // the same per-channel device budget the server would give the channel
            uint64_t ring = 0;
            if (cfg->server_cfg && cfg->server_cfg->ring_blocks)
                ring = cfg->server_cfg->ring_blocks;
            else
                ring = std::max<uint64_t>(
                    128, (cfg->server_cfg ? cfg->server_cfg->ring_bytes : (4ull << 20)) / ch[c]->nb);
            p.device_bytes_cap = ring * ch[c]->nb;
            rc = ext_create(cfg->n_bits[c], cfg->m_bits[c], &p, &ch[c]->ctx);
            if (rc == EXT_OK) rc = ext_stream_open(ch[c]->ctx, 0, 0, &ch[c]->st);
        }
    }
    auto teardown = [&] {
        if (srv) ext_server_destroy(srv);
        for (auto& c : ch)
            if (c->ctx) ext_destroy(c->ctx);
    };
    if (rc != EXT_OK) {
        teardown();
        return rc;
    }

    // ---- run ----------------------------------------------------------------
    const uint64_t t0 = now_ns() + 20000000ull;  // start 20 ms from now
    const uint64_t win_lo = t0 + (uint64_t)(cfg->warmup_s * 1e9);
    const uint64_t win_hi = t0 + (uint64_t)(horizon * 1e9);
    std::atomic<bool> producer_done{false};
    std::atomic<int> fail{EXT_OK};
    std::atomic<uint64_t> eagain{0}, max_lag{0}, chunks_done{0};
    std::atomic<uint64_t> unsubmitted_in_window{0};  // blocks of chunks never submitted
    const uint64_t lag_limit = cfg->max_lag_s > 0 ? (uint64_t)(cfg->max_lag_s * 1e9) : ~0ull;
    const uint32_t n_prod = cfg->producer_threads ? cfg->producer_threads : 4;
    std::atomic<uint32_t> producers_left{n_prod};

    // latencies in 1 us bins up to ~1 s (a fixed histogram never reallocates,
    // so the bookkeeping never stalls the threads that share a channel's lock)
    constexpr uint64_t kBins = 1u << 20;
    std::vector<std::vector<uint32_t>> lag_hist(n_prod, std::vector<uint32_t>(kBins, 0));
    std::vector<uint64_t> lag_n(n_prod, 0);

    // producer p submits the chunks of channels c with c % n_prod == p, in time order
    auto produce = [&](uint32_t pid) {
        size_t next = 0;
        for (; next < ev.size(); ++next) {
            const Event& e = ev[next];
            if (e.ch % n_prod != pid) continue;
            if (fail.load()) break;
            const uint64_t target = t0 + e.t_ns;
            const uint64_t t_now = now_ns();
            if (t_now > target && t_now - target > lag_limit) break;
            for (;;) {
                const uint64_t t = now_ns();
                if (t >= target) break;
                if (target - t > 300000)
                    std::this_thread::sleep_for(std::chrono::nanoseconds(target - t - 200000));
            }
            Chan& c = *ch[e.ch];
            const uint64_t len = (uint64_t)e.k * c.nb;
            // the pool is read cyclically: a chunk that runs past its end goes
            // in two submissions (both whole blocks), the second from the start
            const uint64_t pool = cfg->pool_bytes[e.ch];
            const uint64_t first = std::min(len, pool - c.pool_pos);
            for (int piece = 0; piece < 2 && !fail.load(); ++piece) {
                const uint64_t off = piece ? 0 : c.pool_pos;
                const uint64_t plen = piece ? len - first : first;
                if (!plen) continue;
                const uint8_t* xs = cfg->pool_x[e.ch] + off;
                const uint8_t* ys = cfg->pool_y[e.ch] + off;
                for (;;) {
                    int r;
                    if (srv) {
                        r = ext_server_submit(srv, c.sid, xs, plen, ys, plen);
                    } else {
                        std::lock_guard<std::mutex> g(c.mu);
                        r = ext_submit(c.st, xs, plen, ys, plen, nullptr);
                    }
                    if (r == EXT_EAGAIN) {
                        eagain++;
                        if (now_ns() > win_hi + (uint64_t)(cfg->grace_s * 1e9)) {
                            fail.store(EXT_EAGAIN);
                            break;
                        }
                        std::this_thread::yield();
                        continue;
                    }
                    if (r != EXT_OK) fail.store(r);
                    break;
                }
            }
            if (fail.load()) break;
            const uint64_t t_sub = now_ns();
            const uint64_t lag = t_sub - target;
            if (target >= win_lo && target < win_hi) {
                lag_hist[pid][std::min<uint64_t>(lag / 1000, kBins - 1)] += 1;
                lag_n[pid] += 1;
            }
            uint64_t prev = max_lag.load();
            while (lag > prev && !max_lag.compare_exchange_weak(prev, lag)) {
            }
            c.pool_pos = (c.pool_pos + len) % pool;
            {
                std::lock_guard<std::mutex> g(c.mu);
                c.submitted += e.k;
                c.chunks.push_back(Chan::Rec{c.submitted, target, t_sub});
            }
            chunks_done++;
        }
        uint64_t left = 0;
        for (; next < ev.size(); ++next) {
            if (ev[next].ch % n_prod != pid) continue;
            const uint64_t target = t0 + ev[next].t_ns;
            if (target >= win_lo && target < win_hi) left += ev[next].k;
        }
        unsubmitted_in_window += left;
        if (--producers_left == 0) producer_done.store(true);
    };
    std::vector<std::thread> producers;
    for (uint32_t pidx = 0; pidx < n_prod; ++pidx) producers.emplace_back(produce, pidx);

    // latencies of blocks arrived in the window (exact maximum and sum kept
    // aside), and their service part: from the submission's return to the poll
    std::vector<uint32_t> hist(kBins, 0), svc_hist(kBins, 0), rdy_hist(kBins, 0);
    uint64_t lat_n = 0, lat_max = 0;
    double lat_sum = 0;
    double out_bits = 0, in_bits = 0;
    std::thread consumer([&] {
        uint64_t maxqb = 0;
        for (auto& c : ch) maxqb = std::max(maxqb, c->qb);
        std::vector<uint8_t> buf(maxqb * 256);
        const uint64_t deadline_after = (uint64_t)(cfg->grace_s * 1e9);
        uint64_t producer_end = 0;
        std::vector<uint32_t> ready(nc);
        std::vector<std::pair<uint64_t, uint64_t>> arrivals;  // (arrival, submitted)
        arrivals.reserve(buf.size());
        std::vector<uint64_t> ready_at(buf.size(), 0);  // served mode: when each block was ready
        for (;;) {
            bool progress = false;
            uint32_t n_ready = nc;
            if (srv) {
                // sleep until some channel has output, then visit only those
                const int r = ext_server_ready(srv, ready.data(), nc, &n_ready, 200);
                if (r != EXT_OK) {
                    fail.store(r);
                    break;
                }
            } else {
                for (uint32_t i = 0; i < nc; ++i) ready[i] = i;
            }
            for (uint32_t ri = 0; ri < n_ready && !fail.load(); ++ri) {
                const uint32_t ci = ready[ri];
                Chan& c = *ch[ci];
                size_t len = 0;
                int r;
                const size_t cap = buf.size() / c.qb * c.qb;
                if (srv) {
                    r = ext_server_poll(srv, c.sid, buf.data(), cap, &len, ready_at.data(),
                                        nullptr);
                } else {
                    std::lock_guard<std::mutex> g(c.mu);
                    r = ext_poll(c.st, buf.data(), cap, &len, nullptr);
                }
                if (r != EXT_OK) {
                    fail.store(r);
                    break;
                }
                if (!len) continue;
                const uint64_t t = now_ns();
                progress = true;
                const uint64_t nblk = len / c.qb;
                // arrival time of each returned block: the chunk that completed it
                arrivals.clear();
                {
                    std::lock_guard<std::mutex> g(c.mu);
                    for (uint64_t i = 0; i < nblk; ++i) {
                        const uint64_t blk = c.returned + i;
                        while (!c.chunks.empty() && c.chunks.front().end <= blk)
                            c.chunks.pop_front();
                        if (c.chunks.empty()) break;  // cannot happen: outputs follow submissions
                        arrivals.emplace_back(c.chunks.front().arrival, c.chunks.front().submitted);
                    }
                }
                for (size_t ai = 0; ai < arrivals.size(); ++ai) {
                    const uint64_t arr = arrivals[ai].first, sub = arrivals[ai].second;
                    if (arr < win_lo || arr >= win_hi) continue;
                    const uint64_t l = t - arr;
                    hist[std::min<uint64_t>(l / 1000, kBins - 1)] += 1;
                    svc_hist[std::min<uint64_t>((t - std::min(t, sub)) / 1000, kBins - 1)] += 1;
                    if (srv) {
                        const uint64_t rd = ready_at[ai];
                        rdy_hist[std::min<uint64_t>((rd - std::min(rd, sub)) / 1000, kBins - 1)] += 1;
                    }
                    lat_n += 1;
                    lat_sum += (double)l;
                    lat_max = std::max(lat_max, l);
                    out_bits += 8.0 * c.qb;
                    in_bits += 16.0 * c.nb;
                }
                std::lock_guard<std::mutex> g(c.mu);
                if (cfg->capture && cfg->capture[ci] && cfg->capture_cap) {
                    const uint64_t room = cfg->capture_cap[ci] - c.captured;
                    const uint64_t k = std::min<uint64_t>(room, len);
                    memcpy(cfg->capture[ci] + c.captured, buf.data(), k);
                    c.captured += k;
                }
                c.returned += nblk;
            }
            if (fail.load()) break;
            if (producer_done.load()) {
                if (!producer_end) producer_end = now_ns();
                bool all = true;
                for (auto& cp : ch) {
                    std::lock_guard<std::mutex> g(cp->mu);
                    if (cp->returned < cp->submitted) {
                        all = false;
                        break;
                    }
                }
                if (all || now_ns() > producer_end + deadline_after) break;
            }
            if (!progress) std::this_thread::yield();
        }
    });
    for (auto& t : producers) t.join();
    consumer.join();

    // blocks that arrived in the window but never came back
    uint64_t missing = unsubmitted_in_window.load();
    for (auto& c : ch) {
        std::lock_guard<std::mutex> g(c->mu);
        uint64_t prev_end = 0;
        for (auto& ck : c->chunks) {
            const uint64_t first = std::max(prev_end, c->returned);
            if (ck.arrival >= win_lo && ck.arrival < win_hi && ck.end > first)
                missing += ck.end - first;
            prev_end = ck.end;
        }
    }
    if (srv) {
        ext_server_stats st;
        if (ext_server_stats_get(srv, &st) == EXT_OK) {
            res->cycles = st.cycles;
            res->eagain_ring = st.eagain_ring;
            res->eagain_stage = st.eagain_stage;
            res->mean_cycle_us = st.cycles ? st.gpu_busy_ns / 1e3 / st.cycles : 0.0;
            res->mean_build_us = st.cycles ? st.build_ns / 1e3 / st.cycles : 0.0;
            res->mean_launch_us = st.cycles ? st.launch_ns / 1e3 / st.cycles : 0.0;
            res->max_cycle_us = st.max_cycle_ns / 1e3;
            res->mean_gpu_us = st.cycles ? st.gpu_ns / 1e3 / st.cycles : 0.0;
            res->mean_tiles = st.cycles ? (double)st.tiles / st.cycles : 0.0;
            res->mean_stage_us = st.cycles ? st.stage_ns / 1e3 / st.cycles : 0.0;
            res->mean_extract_us = st.cycles ? st.extract_ns / 1e3 / st.cycles : 0.0;
            res->rings_bytes = st.rings_bytes;
            res->free_bytes = st.free_bytes;
            res->eagain_mem = st.eagain_mem;
        }
    }
    if (capture_len)
        for (uint32_t c = 0; c < nc; ++c) capture_len[c] = ch[c]->captured;
    teardown();
    const int f = fail.load();
    if (f != EXT_OK && f != EXT_EAGAIN) return f;

    res->window_s = cfg->duration_s;
    res->out_gbps = out_bits / cfg->duration_s / 1e9;
    res->in_gbps = in_bits / cfg->duration_s / 1e9;
    res->offered_in_gbps = offered_bits / cfg->duration_s / 1e9;
    res->blocks_measured = lat_n + missing;
    res->blocks_missing = missing;
    res->chunks = chunks_done.load();
    res->eagain = eagain.load();
    res->max_submit_lag_us = max_lag.load() / 1e3;
    // percentile = upper edge of the 1 us bin holding the rank-th value (the
    // last bin also holds everything longer)
    auto pct = [&](const std::vector<uint32_t>& h, uint64_t n, double q) {
        const uint64_t rank = (uint64_t)(q * (double)(n - 1)) + 1;
        uint64_t acc = 0;
        for (uint64_t b = 0; b < kBins; ++b) {
            acc += h[b];
            if (acc >= rank) return (double)(b + 1);
        }
        return (double)kBins;
    };
    if (lat_n) {
        res->lat_p50_us = std::min(pct(hist, lat_n, 0.50), lat_max / 1e3);
        res->lat_p99_us = std::min(pct(hist, lat_n, 0.99), lat_max / 1e3);
        res->lat_max_us = lat_max / 1e3;
        res->lat_mean_us = lat_sum / lat_n / 1e3;
        res->service_p50_us = pct(svc_hist, lat_n, 0.50);
        res->service_p99_us = pct(svc_hist, lat_n, 0.99);
        if (srv) {
            res->ready_p50_us = pct(rdy_hist, lat_n, 0.50);
            res->ready_p99_us = pct(rdy_hist, lat_n, 0.99);
        }
    }
    {
        std::vector<uint32_t> all(kBins, 0);
        uint64_t n = 0;
        for (uint32_t pidx = 0; pidx < n_prod; ++pidx) {
            n += lag_n[pidx];
            for (uint64_t b = 0; b < kBins; ++b) all[b] += lag_hist[pidx][b];
        }
        if (n) res->submit_lag_p99_us = pct(all, n, 0.99);
    }
    return f == EXT_EAGAIN ? EXT_EAGAIN : EXT_OK;
}
