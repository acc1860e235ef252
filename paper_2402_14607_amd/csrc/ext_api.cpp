// ext_api.cpp -- the C ABI (include/qrng_ext.h): contexts, the plain form,
// the streaming form (pending partial blocks kept on the device) and the
// launch planning of the extraction kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/qrng_ext.h"
#include "ext_internal.h"
#include "gf2_modulus.h"

namespace qext {

namespace {
// base-product sizes (words) with a kernel instantiation
bool base_instantiated(uint32_t bw) {
    return (bw >= 1 && bw <= 9) || bw == 11 || bw == 13 || bw == 15 || bw == 16;
}
}  // namespace

bool plan_shape(uint32_t q, uint32_t n_e, const uint32_t* taps, uint32_t n_taps,
                const PlanKnobs& knobs, ExtShape* s) {
    if (q == 0 || q % 8 || n_e == 0 || (n_taps != 1 && n_taps != 3)) return false;
    if ((uint64_t)n_e * q / 8 > 0xffffffffull) return false;
    const uint32_t target = knobs.base_words ? knobs.base_words : 8u;
    if (target > (uint32_t)kMaxBaseWords) return false;
    // Word-aligned elements are multiplied in place when their word count has
    // an odd part the base products cover (<= 15, or knobs.max_odd).  Otherwise (q not a
    // multiple of 32, or such a word count, or asked for) elements are
    // computed in zero-padded slots of qw words, the least count >= q/32
    // whose odd part is covered: the product of padded operands is the same
    // polynomial.
    const uint32_t max_odd = knobs.max_odd ? knobs.max_odd : 15u;
    if (max_odd > 15u) return false;
    auto odd_ok = [&](uint32_t w) { return (w >> __builtin_ctz(w)) <= max_odd; };
    uint32_t qw = (q + 31) / 32;
    const bool padded = (q % 32) != 0 || knobs.padded != 0 || !odd_ok(qw);
    while (!odd_ok(qw)) ++qw;
    const uint32_t v = (uint32_t)__builtin_ctz(qw);
    const uint32_t odd = qw >> v;
    // base size: odd * 2^k words, the largest instantiated one not above the
    // target (or the odd part itself when that is already larger)
    uint32_t bw = odd, levels = v;
    for (uint32_t k = 0; k <= v; ++k) {
        const uint32_t cand = odd << k;
        if (cand > target && k > 0) break;
        if (base_instantiated(cand)) {
            bw = cand;
            levels = v - k;
        }
    }
    if (!base_instantiated(bw) || levels > 10) return false;
    uint32_t max_tap = 0;
    for (uint32_t t = 0; t < n_taps; ++t) {
        if (taps[t] == 0 || taps[t] >= q) return false;
        max_tap = std::max(max_tap, taps[t]);
    }
    if (2 * max_tap > q) return false;  // two folding passes suffice up to q/2
    // element groups: g groups of ceil(n_e / g) elements (the last may hold
    // fewer), for every g that this partition realises exactly
    auto realised = [&](uint32_t g) { return (n_e + (n_e + g - 1) / g - 1) / ((n_e + g - 1) / g) == g; };
    if (knobs.groups && (knobs.groups > n_e || !realised(knobs.groups))) return false;
    const uint32_t threads = knobs.threads ? knobs.threads : (uint32_t)kThreads;
    if (threads % 64 || threads > (uint32_t)kMaxThreads) return false;

    ExtShape r{};
    r.q = q;
    r.qw = qw;
    r.n_e = n_e;
    r.nw = qw * n_e;
    r.padded = padded ? 1u : 0u;
    r.qbytes = q / 8;
    r.nbytes = (uint32_t)((uint64_t)n_e * q / 8);
    r.bw = bw;
    r.levels = levels;
    r.np = 1;
    for (uint32_t l = 0; l < levels; ++l) r.np *= 3;
    r.n_taps = n_taps;
    for (uint32_t t = 0; t < 3; ++t) r.taps[t] = t < n_taps ? taps[t] : 0;
    r.dn = max_tap >= 2 ? (max_tap - 1 + 31) / 32 : 0;

    // Element grouping and pairs per work-group: keep the most lanes busy
    // with the LDS footprint under kMaxLdsBytes (unless fixed by the knobs).
    double best_util = -1.0;
    for (uint32_t stage_try = (levels > 0 || padded) ? 1u : 0u;; stage_try = 0) {
        for (uint32_t g = 1; g <= n_e; ++g) {
            if (!realised(g) || (knobs.groups && g != knobs.groups)) continue;
            const uint32_t per_pair = r.np * g;
            uint32_t ppw = per_pair >= threads ? 1u : threads / per_pair;
            if (knobs.ppw) ppw = knobs.ppw;
            auto lds_words = [&](uint32_t pp) {  // padded shapes add C >> q per pair
                return pp * ((stage_try ? 2 * r.nw : 0) + 2 * qw + r.dn + (padded ? qw : 0)) +
                       (padded ? 2 * kPadSlack : 0);
            };
            // padded staging holds at most kPadRegs slot words per lane
            auto regs_ok = [&](uint32_t pp) {
                return !padded || (uint64_t)pp * r.nw <= (uint64_t)kPadRegs * threads;
            };
            // (a pair count fixed by the knobs may use up to the 64 KiB limit)
            const uint64_t lds_cap = knobs.ppw ? 65536u : kMaxLdsBytes;
            while (ppw > 1 && ((uint64_t)lds_words(ppw) * 4 > lds_cap || !regs_ok(ppw))) --ppw;
            // (unpadded shapes add their rank-major padding, see group_lds_bytes)
            const uint32_t pad = padded ? 0u : ppw * (1u + (stage_try ? 8u : 0u));
            if ((lds_words(ppw) + pad) * 4 > 65536 || !regs_ok(ppw)) continue;
            const uint64_t items = (uint64_t)ppw * per_pair;
            const uint64_t rounds = (items + threads - 1) / threads;
            const double util = (double)items / (double)(rounds * threads);
            if (util > best_util + 1e-9) {
                best_util = util;
                r.groups = g;
                r.epg = (n_e + g - 1) / g;
                r.ppw = ppw;
                r.stage = stage_try;
                r.lds_words = lds_words(ppw);
            }
        }
        if (best_util >= 0 || stage_try == 0 || padded) break;  // padded shapes are staged
    }
    if (best_util < 0) return false;
    r.align = padded ? 1u : (!r.stage && bw % 4 == 0) ? 16u : 4u;
    r.threads = threads;
    *s = r;
    return true;
}

}  // namespace qext

using qext::ExtShape;

// ---------------------------------------------------------------------------
// context and stream objects
// ---------------------------------------------------------------------------
struct ext_ctx {
    uint64_t n_bits = 0;
    uint32_t m_bits = 0;
    uint32_t b = 8;
    std::vector<uint32_t> taps;  // non-leading nonzero exponents, decreasing
    ExtShape shape{};
    // latency plans for launches that would leave CUs idle: one element per
    // lane item and one or more Karatsuba levels beyond the default, so a
    // lane's chain is one short base product (word-level kernel only; same
    // outputs); small[0] has half the default base, each next one half the
    // base before it
    static constexpr uint32_t kMaxSmall = 4;
    ExtShape small[kMaxSmall]{};
    uint32_t n_small = 0;
    uint32_t cus = 0;
    bool bitslice = false;  // plain/streaming launches take the bit-sliced kernel
    uint32_t kernel = EXT_KERNEL_AUTO;  // ext_params.kernel, for streams of other shapes
    uint32_t mem_kind = EXT_MEM_HOST;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t copy_stream = nullptr;  // D2H copies of finished outputs
    int device = 0;
    uint64_t cap = 0;
    int sticky = EXT_OK;
    // device scratch for host-memory ext_extract
    uint8_t* dx = nullptr;
    uint8_t* dy = nullptr;
    uint8_t* dout = nullptr;
    uint64_t scratch_pairs = 0;
    std::vector<ext_stream*> streams;
};

namespace {

struct Launch {
    uint64_t ring_pos;  // first output slot in the stream's output ring
    uint64_t n;         // block pairs
    uint64_t consumed;  // pairs already handed out by ext_poll
    hipEvent_t done;
};

}  // namespace

struct ext_stream {
    ext_ctx* ctx = nullptr;
    bool closed = false;
    uint64_t nb = 0;  // bytes per block
    uint64_t qb = 0;  // output bytes per block
    ExtShape shape{};       // launch plan of the stream's (n, m)
    bool bitslice = false;  // the stream's launches take the bit-sliced kernel
    // pending input on the device: double buffers, live bytes [head, tail)
    uint8_t* xbuf[2] = {nullptr, nullptr};
    uint8_t* ybuf[2] = {nullptr, nullptr};
    int xcur = 0, ycur = 0;
    uint64_t buf_bytes = 0;
    uint64_t xhead = 0, xtail = 0, yhead = 0, ytail = 0;
    // outputs: ring of out_slots block outputs
    uint8_t* oring = nullptr;
    uint64_t out_slots = 0;
    uint64_t ring_write = 0;  // next slot to fill (monotonic, mod out_slots)
    uint64_t ring_used = 0;   // slots launched but not yet polled
    std::deque<Launch> inflight;
    uint64_t launched = 0;
    uint64_t returned = 0;
    // pinned staging for host submissions
    uint8_t* stage = nullptr;
    uint64_t stage_bytes = 0;
    hipEvent_t stage_free = nullptr;
};

namespace {

int fail(ext_ctx* c, hipError_t e) {
    if (e == hipSuccess) return EXT_OK;
    if (c) c->sticky = EXT_EDEVICE;
    return EXT_EDEVICE;
}

#define HIP_TRY(ctx, expr)                          \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return fail(ctx, _e); \
    } while (0)

int enter(ext_ctx* c) {
    if (!c) return EXT_EINVAL;
    if (c->sticky) return c->sticky;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(c, hipErrorInvalidDevice);
    if (cur != c->device && hipSetDevice(c->device) != hipSuccess)
        return fail(c, hipErrorInvalidDevice);
    return EXT_OK;
}

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

int launch(ext_ctx* c, const ExtShape& shape, bool bitslice, const void* x, const void* y,
           void* out, uint64_t n_pairs) {
    if (bitslice)
        HIP_TRY(c, qext::launch_bitslice(shape, (const uint8_t*)x, (const uint8_t*)y,
                                         (uint8_t*)out, n_pairs, c->stream));
    else
        HIP_TRY(c, qext::launch_extract(shape, (const uint8_t*)x, (const uint8_t*)y,
                                        (uint8_t*)out, n_pairs, c->stream));
    return EXT_OK;
}

int launch(ext_ctx* c, const void* x, const void* y, void* out, uint64_t n_pairs) {
    if (!c->bitslice && c->n_small) {
        // fewer work-groups than CUs: a latency plan spreads the same pairs
        // over more of them, each lane one base product; the smallest base
        // whose launch stays within two work-groups per CU (smaller bases do
        // more work in all, which a fuller GPU would pay for), else the
        // half-size base
        const uint64_t wgs = (n_pairs + c->shape.ppw - 1) / c->shape.ppw;
        if (wgs < c->cus) {
            for (uint32_t i = c->n_small; i-- > 0;) {
                const ExtShape& sm = c->small[i];
                const uint64_t w = (n_pairs + sm.ppw - 1) / sm.ppw;
                if (w > wgs && (w <= 2ull * c->cus || i == 0))
                    return launch(c, sm, false, x, y, out, n_pairs);
            }
        }
    }
    return launch(c, c->shape, c->bitslice, x, y, out, n_pairs);
}

// The bit-sliced kernel applies to fields up to kBitsliceMaxQ bits and
// blocks below 8 MiB (its chunked planes stay below 64 KiB of LDS).
bool bitslice_applies(const ExtShape& s) {
    uint32_t max_tap = 0;  // its reduction folds twice, which suffices up to q/2
    for (uint32_t k = 0; k < s.n_taps; ++k) max_tap = std::max(max_tap, s.taps[k]);
    return s.q <= qext::kBitsliceMaxQ && s.q % 8 == 0 && s.nbytes < (1u << 23) &&
           2 * max_tap <= s.q && (uint64_t)qext::bitslice_lds_words(s) * 4 <= 65536;
}

// EXT_KERNEL_AUTO's choice without autotuning, among the shapes the
// bit-sliced kernel applies to: enough elements per block to amortize its
// per-group end phase.  Measured on MI355X over q = 16 .. 128 (step 8) and
// n_e in {2, 4, 8, 16, 30, 71, 150}: at the counts at or above these it was
// 1.17-3.8x as fast as the word-level kernel, below them 0.15-1.14x; fields
// that are whole 32-bit words (which the word-level kernel takes unpadded)
// need the most elements.
bool bitslice_preferred(const ExtShape& s) {
    if (s.q < 16 || s.q > 128 || s.q % 8) return false;
    uint32_t min_ne;
    if (s.q == 32) min_ne = 100;
    else if (s.q % 32 == 0) min_ne = 64;  // 64, 96, 128
    else if (s.q < 40) min_ne = 40;   // 16, 24
    else if (s.q < 64) min_ne = 24;   // 40, 48, 56
    else min_ne = 16;                 // 72 .. 120 except 96
    return s.n_e >= min_ne;
}

// The launch plan of (n_bits, m_bits, taps) for ext_params.kernel `kernel`
// without autotuning: the word-level plan from the knobs, and whether the
// bit-sliced kernel takes the shape (the AUTO rule, or asked for).  *bsh
// receives the bit-sliced kernel's shape, *bs_ok whether it applies.
// EXT_ENOTSUP when no kernel takes the shape.
int plan_kernel(uint64_t n_bits, uint32_t m_bits, const std::vector<uint32_t>& taps,
                const qext::PlanKnobs& knobs, uint32_t kernel, ExtShape* shape, bool* bitslice,
                ExtShape* bsh, bool* bs_ok) {
    const uint32_t n_e = (uint32_t)(n_bits / m_bits);
    const bool planned = qext::plan_shape(m_bits, n_e, taps.data(), (uint32_t)taps.size(), knobs,
                                          shape);
    bool bs = false, ok = false;
    *bsh = ExtShape{};
    if (kernel != EXT_KERNEL_WORD) {
        bsh->q = m_bits;
        bsh->n_e = n_e;
        bsh->n_taps = (uint32_t)taps.size();
        for (size_t k = 0; k < taps.size(); ++k) bsh->taps[k] = taps[k];
        bsh->qbytes = m_bits / 8;
        bsh->nbytes = (uint32_t)(n_bits / 8);
        bsh->align = 1;  // byte gathers
        bsh->threads = qext::kThreads;
        ok = m_bits % 8 == 0 && n_bits / 8 < (1ull << 23) && bitslice_applies(*bsh);
        bs = ok && (kernel == EXT_KERNEL_BITSLICE || !planned || bitslice_preferred(*bsh));
    }
    if (kernel == EXT_KERNEL_BITSLICE && !bs) return EXT_ENOTSUP;
    if (!bs && !planned) return EXT_ENOTSUP;
    if (bs) {
        if (planned) shape->align = 1;  // byte gathers
        else *shape = *bsh;
    }
    *bitslice = bs;
    *bs_ok = ok && planned;
    return EXT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void ext_params_init(ext_params* p) {
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->sample_bits = 8;
    p->mem_kind = EXT_MEM_HOST;
    p->device_bytes_cap = 256ull << 20;
    p->device = -1;
}

const char* ext_strerror(int code) {
    switch (code) {
        case EXT_OK: return "ok";
        case EXT_EINVAL: return "invalid argument";
        case EXT_ENOTSUP: return "shape or modulus not supported by the GPU path";
        case EXT_ENOMEM: return "out of memory";
        case EXT_EAGAIN: return "device buffer full (admission): poll and retry";
        case EXT_EDEVICE: return "HIP device error";
        case EXT_ECLOSED: return "stream closed";
        default: return "unknown status";
    }
}

int ext_is_irreducible(uint32_t m_bits, const uint32_t* taps, uint32_t n_taps) {
    if (m_bits < 2 || (n_taps && !taps) || n_taps > 3) return EXT_EINVAL;
    for (uint32_t k = 0; k < n_taps; ++k)
        if (taps[k] == 0 || taps[k] >= m_bits) return EXT_EINVAL;
    return qext::modulus_is_irreducible(m_bits, taps, n_taps) ? 1 : 0;
}

int ext_default_modulus(uint32_t m_bits, uint32_t* exps, uint32_t cap, uint32_t* n) {
    if (!exps || !n || m_bits < 2) return EXT_EINVAL;
    std::vector<uint32_t> taps;
    try {
        if (!qext::default_modulus(m_bits, &taps)) return EXT_ENOTSUP;
    } catch (const std::bad_alloc&) {
        return EXT_ENOMEM;
    }
    if (cap < taps.size() + 2) return EXT_EINVAL;
    uint32_t k = 0;
    exps[k++] = m_bits;
    for (uint32_t t : taps) exps[k++] = t;
    exps[k++] = 0;
    *n = k;
    return EXT_OK;
}

int ext_create(uint64_t n_bits, uint32_t m_bits, const ext_params* p, ext_ctx** out) {
    if (!out) return EXT_EINVAL;
    *out = nullptr;
    ext_params def;
    ext_params_init(&def);
    if (!p) p = &def;
    const uint32_t b = p->sample_bits ? p->sample_bits : 8;
    if (n_bits == 0 || m_bits == 0 || n_bits % m_bits || m_bits % b) return EXT_EINVAL;
    if (p->mem_kind != EXT_MEM_HOST && p->mem_kind != EXT_MEM_DEVICE) return EXT_EINVAL;
    if (n_bits / m_bits > 0xffffffffull) return EXT_EINVAL;
    if (p->kernel > EXT_KERNEL_BITSLICE) return EXT_EINVAL;
    std::vector<uint32_t> taps;
    if (p->n_taps == 0) {
        try {
            if (!qext::default_modulus(m_bits, &taps)) return EXT_ENOTSUP;
        } catch (const std::bad_alloc&) {
            return EXT_ENOMEM;
        }
    } else if (p->n_taps == 1 || p->n_taps == 3) {
        taps.assign(p->taps, p->taps + p->n_taps);
        std::sort(taps.begin(), taps.end(), std::greater<uint32_t>());
        for (size_t k = 0; k < taps.size(); ++k) {
            if (taps[k] == 0 || taps[k] >= m_bits) return EXT_EINVAL;
            if (k && taps[k] == taps[k - 1]) return EXT_EINVAL;
        }
        if (!qext::modulus_is_irreducible(m_bits, taps.data(), (uint32_t)taps.size()))
            return EXT_EINVAL;
    } else {
        return EXT_EINVAL;
    }
    ExtShape shape, bsh;
    qext::PlanKnobs knobs{p->base_bits / 32, p->groups, p->pairs_per_group, p->threads};
    if (p->base_bits % 32) return EXT_EINVAL;
    bool bs = false, bs_ok = false;
    const int prc = plan_kernel(n_bits, m_bits, taps, knobs, p->kernel, &shape, &bs, &bsh, &bs_ok);
    if (prc) return prc;
    // AUTO with autotune: a timing once the stream exists decides
    const bool tune_kernel = bs_ok && p->kernel == EXT_KERNEL_AUTO && p->autotune;
    ext_ctx* c = new (std::nothrow) ext_ctx;
    if (!c) return EXT_ENOMEM;
    c->bitslice = bs;
    c->kernel = p->kernel;
    c->n_bits = n_bits;
    c->m_bits = m_bits;
    c->b = b;
    c->taps = taps;
    c->shape = shape;
    c->mem_kind = p->mem_kind;
    c->cap = p->device_bytes_cap ? p->device_bytes_cap : (256ull << 20);
    int dev = p->device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        delete c;
        return EXT_EDEVICE;
    }
    c->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
        delete c;
        return EXT_EDEVICE;
    }
    if (p->use_hip_stream) {
        c->stream = (hipStream_t)p->hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return EXT_EDEVICE;
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return EXT_EDEVICE;
    }
    if (tune_kernel) {
        bool use_bs = false;
        if (qext::choose_kernel(bsh, c->stream, &use_bs) != hipSuccess) {
            (void)hipStreamDestroy(c->copy_stream);
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return EXT_EDEVICE;
        }
        c->bitslice = use_bs;
        if (use_bs) c->shape.align = 1;
    }
    if (p->autotune && !c->bitslice) {
        qext::PlanKnobs tuned;
        ExtShape ts;
        if (qext::autotune_shape(m_bits, (uint32_t)(n_bits / m_bits), taps.data(),
                                 (uint32_t)taps.size(), c->stream, &tuned, nullptr) != hipSuccess ||
            !qext::plan_shape(m_bits, (uint32_t)(n_bits / m_bits), taps.data(),
                              (uint32_t)taps.size(), tuned, &ts)) {
            (void)hipStreamDestroy(c->copy_stream);
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return EXT_EDEVICE;
        }
        c->shape = ts;
    }
    // the latency plan (when the caller fixed no plan knob): every element
    // its own lane item, base half the default's (one more Karatsuba level),
    // halved again while a pair's items (n_e * 3^levels) still fit in one
    // round of the group's lanes, so that each lane's chain is one shorter
    // base product; a base whose items need a second round is not taken
    if (!c->bitslice && !p->base_bits && !p->groups && !p->pairs_per_group) {
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const ExtShape& d = c->shape;
        // (inputs are checked against the default plan's alignment, which
        // the latency plan's must divide)
        auto small_plan = [&](uint32_t bw, ExtShape* ss) {
            const qext::PlanKnobs sk{bw, d.n_e, 0, d.threads, d.padded};
            return qext::plan_shape(m_bits, d.n_e, taps.data(), (uint32_t)taps.size(), sk, ss) &&
                   ss->padded == d.padded && ss->qw == d.qw && d.align % ss->align == 0;
        };
        auto one_round = [](const ExtShape& ss) {
            return (uint64_t)ss.np * ss.groups <= ss.threads;
        };
        uint32_t bw = d.bw > 1 ? d.bw / 2 : 1;
        ExtShape ss;
        if (cus > 0 && small_plan(bw, &ss)) {
            c->small[0] = ss;
            c->n_small = 1;
            while (bw > 1 && c->n_small < ext_ctx::kMaxSmall && one_round(ss)) {
                ExtShape s2;
                if (!small_plan(bw / 2, &s2) || !one_round(s2)) break;
                bw /= 2;
                if (s2.bw == ss.bw) continue;  // the base target rounded to the same size
                ss = s2;
                c->small[c->n_small++] = ss;
            }
            c->cus = (uint32_t)cus;
        }
    }
    *out = c;
    return EXT_OK;
}

int ext_get_modulus(const ext_ctx* c, uint32_t* exps, uint32_t cap, uint32_t* n) {
    if (!c || !exps || !n) return EXT_EINVAL;
    if (cap < c->taps.size() + 2) return EXT_EINVAL;
    uint32_t k = 0;
    exps[k++] = c->m_bits;
    for (uint32_t t : c->taps) exps[k++] = t;
    exps[k++] = 0;
    *n = k;
    return EXT_OK;
}

int ext_describe(const ext_ctx* c, char* buf, size_t cap) {
    if (!c || !buf || cap == 0) return EXT_EINVAL;
    const ExtShape& s = c->shape;
    if (c->bitslice) {
        uint32_t ec = 0, levels = 0, piece = 0, subs = 0;
        qext::bitslice_describe(s, &ec, &levels, &piece, &subs);
        snprintf(buf, cap,
                 "{\"n\": %llu, \"m\": %u, \"n_e\": %u, \"kernel\": \"bitslice\", "
                 "\"pairs_per_workgroup\": 32, \"threads\": %d, \"lds_bytes\": %u, "
                 "\"chunk_elements\": %u, \"karatsuba_levels\": %u, \"piece_planes\": %u, "
                 "\"element_subsets\": %u}",
                 (unsigned long long)c->n_bits, c->m_bits, (uint32_t)(c->n_bits / c->m_bits),
                 qext::kThreads, qext::bitslice_lds_words(s) * 4, ec, levels, piece, subs);
        return EXT_OK;
    }
    // small_launch: the smallest-base latency plan, and the bases of all of them
    char small[256] = "";
    if (c->n_small) {
        const ExtShape& sm = c->small[c->n_small - 1];
        char bases[64] = "";
        size_t used = 0;
        for (uint32_t i = 0; i < c->n_small && used < sizeof bases; ++i)
            used += (size_t)snprintf(bases + used, sizeof bases - used, "%s%u", i ? ", " : "",
                                     c->small[i].bw * 32);
        snprintf(small, sizeof small,
                 ", \"small_launch\": {\"below_workgroups\": %u, \"base_bits\": %u, "
                 "\"karatsuba_levels\": %u, \"pairs_per_workgroup\": %u, \"element_groups\": %u, "
                 "\"bases\": [%s], \"smallest_within_workgroups\": %u}",
                 c->cus, sm.bw * 32, sm.levels, sm.ppw, sm.groups, bases, 2u * c->cus);
    }
    snprintf(buf, cap,
             "{\"n\": %llu, \"m\": %u, \"n_e\": %u, \"base_bits\": %u, \"karatsuba_levels\": %u, "
             "\"subproducts\": %u, \"pairs_per_workgroup\": %u, \"element_groups\": %u, "
             "\"staged\": %u, \"lds_bytes\": %u, \"threads\": %d, \"padded\": %u, "
             "\"slot_words\": %u, \"kernel\": \"%s\"%s}",
             (unsigned long long)c->n_bits, c->m_bits, s.n_e, s.bw * 32, s.levels, s.np, s.ppw,
             s.groups, s.stage, qext::group_lds_bytes(s), s.threads, s.padded, s.qw, "word", small);
    return EXT_OK;
}

int ext_probe_valu_rate(int device, double* lane_ops_per_s) {
    if (!lane_ops_per_s) return EXT_EINVAL;
    *lane_ops_per_s = 0.0;
    int dev = device;
    if ((dev < 0 && hipGetDevice(&dev) != hipSuccess) || hipSetDevice(dev) != hipSuccess)
        return EXT_EDEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return EXT_EDEVICE;
    const uint32_t blocks = (uint32_t)cus * 32u, iters = 1000u;
    uint32_t* out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = EXT_OK;
    float best_ms = 0.f;
    if (hipMalloc((void**)&out, (size_t)blocks * qext::kThreads * 4) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = EXT_EDEVICE;
    }
    // one warm-up run, then the fastest of three
    for (int rep = 0; rep < 4 && rc == EXT_OK; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess ||
            qext::launch_valu_probe(out, blocks, iters, st) != hipSuccess ||
            hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = EXT_EDEVICE;
            break;
        }
        if (rep > 0 && (best_ms == 0.f || ms < best_ms)) best_ms = ms;
    }
    if (rc == EXT_OK && best_ms > 0.f)
        *lane_ops_per_s = (double)blocks * qext::kThreads * iters * qext::kProbeOpsPerIter /
                          (best_ms * 1e-3);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(out);
    (void)hipGetLastError();
    return rc;
}

int ext_sync(ext_ctx* c) {
    int rc = enter(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return EXT_OK;
}

int ext_extract(ext_ctx* c, const void* x, const void* y, uint64_t n_pairs, void* out) {
    int rc = enter(c);
    if (rc) return rc;
    if (n_pairs == 0) return EXT_OK;
    if (!x || !y || !out) return EXT_EINVAL;
    if (!aligned4(x) || !aligned4(y) || !aligned4(out)) return EXT_EINVAL;
    const uint64_t nb = c->n_bits / 8, qb = c->m_bits / 8;
    if (c->mem_kind == EXT_MEM_DEVICE) {
        const uintptr_t am = c->shape.align - 1;
        if (((uintptr_t)x & am) || ((uintptr_t)y & am)) return EXT_EINVAL;
        return launch(c, x, y, out, n_pairs);
    }
    // host memory: stage through device scratch, in slices of at most 64 MiB
    // of input per side
    const uint64_t slice = std::max<uint64_t>(1, (64ull << 20) / nb);
    const uint64_t want = std::min(slice, n_pairs);
    if (c->scratch_pairs < want) {
        (void)hipFree(c->dx);
        (void)hipFree(c->dy);
        (void)hipFree(c->dout);
        c->dx = c->dy = c->dout = nullptr;
        c->scratch_pairs = 0;
        if (hipMalloc((void**)&c->dx, want * nb) != hipSuccess ||
            hipMalloc((void**)&c->dy, want * nb) != hipSuccess ||
            hipMalloc((void**)&c->dout, want * qb) != hipSuccess) {
            (void)hipFree(c->dx);
            (void)hipFree(c->dy);
            (void)hipFree(c->dout);
            c->dx = c->dy = c->dout = nullptr;
            (void)hipGetLastError();
            return EXT_ENOMEM;
        }
        c->scratch_pairs = want;
    }
    for (uint64_t done = 0; done < n_pairs;) {
        const uint64_t k = std::min(c->scratch_pairs, n_pairs - done);
        HIP_TRY(c, hipMemcpyAsync(c->dx, (const uint8_t*)x + done * nb, k * nb,
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->dy, (const uint8_t*)y + done * nb, k * nb,
                                  hipMemcpyHostToDevice, c->stream));
        rc = launch(c, c->dx, c->dy, c->dout, k);
        if (rc) return rc;
        HIP_TRY(c, hipMemcpyAsync((uint8_t*)out + done * qb, c->dout, k * qb,
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        done += k;
    }
    return EXT_OK;
}

int ext_destroy(ext_ctx* c) {
    if (!c) return EXT_OK;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != c->device) (void)hipSetDevice(c->device);
    while (!c->streams.empty()) ext_stream_close(c->streams.back(), nullptr);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->dx);
    (void)hipFree(c->dy);
    (void)hipFree(c->dout);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return EXT_OK;
}

// ---------------------------------------------------------------------------
// streaming form
// ---------------------------------------------------------------------------
int ext_stream_open(ext_ctx* c, uint64_t n_bits, uint32_t m_bits, ext_stream** out) {
    if (!out) return EXT_EINVAL;
    *out = nullptr;
    int rc = enter(c);
    if (rc) return rc;
    if (!n_bits) n_bits = c->n_bits;
    if (!m_bits) m_bits = c->m_bits;
    ExtShape shape = c->shape;
    bool bitslice = c->bitslice;
    if (n_bits != c->n_bits || m_bits != c->m_bits) {
        // a shape of its own: the context's modulus when the field is the
        // context's, else the conventional one of degree m; the default plan
        if (n_bits % m_bits || m_bits % c->b || n_bits / m_bits > 0xffffffffull)
            return EXT_EINVAL;
        std::vector<uint32_t> taps;
        if (m_bits == c->m_bits) {
            taps = c->taps;
        } else {
            try {
                if (!qext::default_modulus(m_bits, &taps)) return EXT_ENOTSUP;
            } catch (const std::bad_alloc&) {
                return EXT_ENOMEM;
            }
        }
        ExtShape bsh;
        bool bs_ok = false;
        rc = plan_kernel(n_bits, m_bits, taps, qext::PlanKnobs{}, c->kernel, &shape, &bitslice,
                         &bsh, &bs_ok);
        if (rc) return rc;
    }
    ext_stream* s = new (std::nothrow) ext_stream;
    if (!s) return EXT_ENOMEM;
    s->ctx = c;
    s->nb = n_bits / 8;
    s->qb = m_bits / 8;
    s->shape = shape;
    s->bitslice = bitslice;
    // every side holds at most cap bytes of pending input plus one block
    s->buf_bytes = ((c->cap + s->nb - 1) / s->nb + 1) * s->nb;
    // room for as many outputs as the pending input could produce, times two
    s->out_slots = 2 * (s->buf_bytes / s->nb);
    bool ok = true;
    for (int k = 0; k < 2 && ok; ++k) {
        ok = hipMalloc((void**)&s->xbuf[k], s->buf_bytes) == hipSuccess &&
             hipMalloc((void**)&s->ybuf[k], s->buf_bytes) == hipSuccess;
    }
    ok = ok && hipMalloc((void**)&s->oring, s->out_slots * s->qb) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->stage_free, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int k = 0; k < 2; ++k) {
            (void)hipFree(s->xbuf[k]);
            (void)hipFree(s->ybuf[k]);
        }
        (void)hipFree(s->oring);
        if (s->stage_free) (void)hipEventDestroy(s->stage_free);
        (void)hipGetLastError();
        delete s;
        return EXT_ENOMEM;
    }
    c->streams.push_back(s);
    *out = s;
    return EXT_OK;
}

namespace {

// Make room for `len` more bytes on one side: compact [head, tail) to the
// front of the other buffer when the tail would run past the end.
int make_room(ext_stream* s, uint8_t** buf, int* cur, uint64_t* head, uint64_t* tail,
              uint64_t len) {
    ext_ctx* c = s->ctx;
    const uint64_t live = *tail - *head;
    if (live + len > s->buf_bytes) return EXT_EAGAIN;
    if (*tail + len <= s->buf_bytes) return EXT_OK;
    const int nxt = 1 - *cur;
    if (live)
        HIP_TRY(c, hipMemcpyAsync(buf[nxt], buf[*cur] + *head, live, hipMemcpyDeviceToDevice,
                                  c->stream));
    *cur = nxt;
    *head = 0;
    *tail = live;
    return EXT_OK;
}

// Queue the copy of one submission (x_len bytes of X, y_len of Y) to the
// tails of the pending buffers.  Host data go through pinned staging, reused
// once the previous submission's copies have completed.
int append(ext_stream* s, const void* x, uint64_t x_len, const void* y, uint64_t y_len) {
    ext_ctx* c = s->ctx;
    uint8_t* xdst = s->xbuf[s->xcur] + s->xtail;
    uint8_t* ydst = s->ybuf[s->ycur] + s->ytail;
    if (c->mem_kind == EXT_MEM_DEVICE) {
        if (x_len)
            HIP_TRY(c, hipMemcpyAsync(xdst, x, x_len, hipMemcpyDeviceToDevice, c->stream));
        if (y_len)
            HIP_TRY(c, hipMemcpyAsync(ydst, y, y_len, hipMemcpyDeviceToDevice, c->stream));
        return EXT_OK;
    }
    if (!x_len && !y_len) return EXT_OK;
    HIP_TRY(c, hipEventSynchronize(s->stage_free));
    const uint64_t len = x_len + y_len;
    if (s->stage_bytes < len) {
        if (s->stage) (void)hipHostFree(s->stage);
        s->stage = nullptr;
        s->stage_bytes = 0;
        if (hipHostMalloc((void**)&s->stage, len, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return EXT_ENOMEM;
        }
        s->stage_bytes = len;
    }
    if (x_len) memcpy(s->stage, x, x_len);
    if (y_len) memcpy(s->stage + x_len, y, y_len);
    if (x_len)
        HIP_TRY(c, hipMemcpyAsync(xdst, s->stage, x_len, hipMemcpyHostToDevice, c->stream));
    if (y_len)
        HIP_TRY(c, hipMemcpyAsync(ydst, s->stage + x_len, y_len, hipMemcpyHostToDevice,
                                  c->stream));
    HIP_TRY(c, hipEventRecord(s->stage_free, c->stream));
    return EXT_OK;
}

int launch_ready(ext_stream* s) {
    ext_ctx* c = s->ctx;
    uint64_t ready = std::min(s->xtail - s->xhead, s->ytail - s->yhead) / s->nb;
    while (ready) {
        if (s->ring_used >= s->out_slots) return EXT_EAGAIN;
        const uint64_t pos = s->ring_write % s->out_slots;
        uint64_t k = std::min(ready, s->out_slots - s->ring_used);
        k = std::min(k, s->out_slots - pos);  // no wrap inside one launch
        const uint8_t* xp = s->xbuf[s->xcur] + s->xhead;
        const uint8_t* yp = s->ybuf[s->ycur] + s->yhead;
        if (((uintptr_t)xp | (uintptr_t)yp) & (s->shape.align - 1)) return EXT_EINVAL;
        int rc = launch(c, s->shape, s->bitslice, xp, yp, s->oring + pos * s->qb, k);
        if (rc) return rc;
        Launch L{pos, k, 0, nullptr};
        HIP_TRY(c, hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
        HIP_TRY(c, hipEventRecord(L.done, c->stream));
        s->inflight.push_back(L);
        s->ring_write += k;
        s->ring_used += k;
        s->launched += k;
        s->xhead += k * s->nb;
        s->yhead += k * s->nb;
        ready -= k;
    }
    return EXT_OK;
}

int copy_out(ext_stream* s, void* out, size_t out_cap, size_t* out_len, uint64_t* blocks_done,
             bool wait) {
    ext_ctx* c = s->ctx;
    size_t written = 0;
    while (!s->inflight.empty()) {
        Launch& L = s->inflight.front();
        if (wait) {
            HIP_TRY(c, hipEventSynchronize(L.done));
        } else {
            hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return fail(c, q);
        }
        const uint64_t avail = L.n - L.consumed;
        const uint64_t fit = (out_cap - written) / s->qb;
        const uint64_t k = std::min(avail, fit);
        if (k) {
            const uint8_t* src = s->oring + (L.ring_pos + L.consumed) * s->qb;
            const hipMemcpyKind kind = c->mem_kind == EXT_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                                     : hipMemcpyDeviceToHost;
            HIP_TRY(c, hipMemcpyAsync((uint8_t*)out + written, src, k * s->qb, kind,
                                      c->copy_stream));
            HIP_TRY(c, hipStreamSynchronize(c->copy_stream));
            written += k * s->qb;
            L.consumed += k;
            s->returned += k;
            s->ring_used -= k;
        }
        if (L.consumed < L.n) break;  // caller's buffer is full
        (void)hipEventDestroy(L.done);
        s->inflight.pop_front();
    }
    if (out_len) *out_len = written;
    if (blocks_done) *blocks_done = s->returned;
    return EXT_OK;
}

}  // namespace

int ext_submit(ext_stream* s, const void* x, size_t x_len, const void* y, size_t y_len,
               uint64_t* seq_out) {
    if (!s) return EXT_EINVAL;
    if (s->closed) return EXT_ECLOSED;
    ext_ctx* c = s->ctx;
    int rc = enter(c);
    if (rc) return rc;
    if ((x_len && !x) || (y_len && !y)) return EXT_EINVAL;
    // admission: pending bytes on each side must stay within the cap
    if ((s->xtail - s->xhead) + x_len > s->buf_bytes ||
        (s->ytail - s->yhead) + y_len > s->buf_bytes)
        return EXT_EAGAIN;
    // outputs that this chunk completes must fit in the output ring
    {
        const uint64_t nx = (s->xtail - s->xhead + x_len) / s->nb;
        const uint64_t ny = (s->ytail - s->yhead + y_len) / s->nb;
        if (s->ring_used + std::min(nx, ny) > s->out_slots) return EXT_EAGAIN;
    }
    rc = make_room(s, s->xbuf, &s->xcur, &s->xhead, &s->xtail, x_len);
    if (rc) return rc;
    rc = make_room(s, s->ybuf, &s->ycur, &s->yhead, &s->ytail, y_len);
    if (rc) return rc;
    rc = append(s, x, x_len, y, y_len);
    if (rc) return rc;
    s->xtail += x_len;
    s->ytail += y_len;
    rc = launch_ready(s);
    if (rc) return rc;
    if (seq_out) *seq_out = s->launched;
    return EXT_OK;
}

int ext_poll(ext_stream* s, void* out, size_t out_cap, size_t* out_len, uint64_t* blocks_done) {
    if (!s) return EXT_EINVAL;
    if (s->closed) return EXT_ECLOSED;
    int rc = enter(s->ctx);
    if (rc) return rc;
    if (!out && out_cap) return EXT_EINVAL;
    return copy_out(s, out, out_cap, out_len, blocks_done, false);
}

int ext_drain(ext_stream* s, void* out, size_t out_cap, size_t* out_len, uint64_t* blocks_done) {
    if (!s) return EXT_EINVAL;
    if (s->closed) return EXT_ECLOSED;
    int rc = enter(s->ctx);
    if (rc) return rc;
    if (!out && out_cap) return EXT_EINVAL;
    return copy_out(s, out, out_cap, out_len, blocks_done, true);
}

int ext_stream_close(ext_stream* s, uint64_t* dropped_bits) {
    if (!s) return EXT_EINVAL;
    ext_ctx* c = s->ctx;
    const uint64_t px = s->xtail - s->xhead, py = s->ytail - s->yhead;
    if (dropped_bits) *dropped_bits = 8 * std::max(px, py);
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != c->device) (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (Launch& L : s->inflight) (void)hipEventDestroy(L.done);
    s->inflight.clear();
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(s->xbuf[k]);
        (void)hipFree(s->ybuf[k]);
    }
    (void)hipFree(s->oring);
    if (s->stage) (void)hipHostFree(s->stage);
    if (s->stage_free) (void)hipEventDestroy(s->stage_free);
    auto it = std::find(c->streams.begin(), c->streams.end(), s);
    if (it != c->streams.end()) c->streams.erase(it);
    s->closed = true;
    delete s;
    return EXT_OK;
}

}  // extern "C"
