// ext_bsk.h -- geometry and index arithmetic of the bit-sliced Karatsuba
// kernel (ext_bsk.hip), shared by the kernel and the host code that plans
// its launches.  Plain C++ with host/device inline functions, no HIP calls.
//
// Fields F_2^q with q = 256 * 2^L, L = 1 .. 3 (q = 512, 1024, 2048).  A
// work-group takes 32 block pairs; bit p of every 32-bit "plane" word belongs
// to pair p.  Element products are split L Karatsuba levels down to 3^L
// products of 256-bit operands (the sub-products), each computed as a
// schoolbook product of bit planes, c[t] ^= x[j] & y[t - j], one AND-XOR per
// (j, t) for all 32 pairs at once -- no shifts and no masks.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define QEXT_HD __host__ __device__
#else
#define QEXT_HD
#endif

namespace qext {

constexpr uint32_t kBskPairs = 32;   // pairs per work-group (bits of a plane)
constexpr uint32_t kBskBase = 256;   // planes per Karatsuba base operand
constexpr uint32_t kBskLeaf = 265;   // LDS words per 256 planes (pad(256))
constexpr uint32_t kBskMaxL = 3;
constexpr uint32_t kBskMaxNp = 27;   // 3^kBskMaxL
constexpr uint32_t kBskIters = 17;   // 16x16 tiles per lane task (two t-blocks)
constexpr uint32_t kBskStage = 3;    // 16-byte staging loads per lane per element

// LDS word of plane j in a plane array: one pad word after every 32 planes,
// so that 32 lanes writing plane 32w + i (lane w) hit 32 different banks, and
// one more after every 256, so that the 256-plane segments (and the operands
// laid out like them) start 265 words apart -- 9 banks on -- and the lanes
// of one task, which read different sub-products' operands, spread over the
// banks.  Within a segment, plane k sits at k + k/32.
QEXT_HD constexpr uint32_t bsk_pad(uint32_t j) { return j + (j >> 5) + (j >> 8); }

// Karatsuba path of sub-product p (one base-3 digit per level: 0 low halves,
// 1 high halves, 2 sum of halves; bit l describes the level whose halves are
// 256 * 2^l planes).  Operand of p: XOR over sub within mid of the 256-plane
// segment (hi | sub).  Product of p: added to the full product at plane
// offsets 256 (hi | mid) + 256 sub' for every sub' within lmask & ~mid.
QEXT_HD inline void bsk_path(uint32_t p, uint32_t levels, uint32_t* hi, uint32_t* mid) {
    uint32_t h = 0, m = 0, v = p;
    for (uint32_t l = 0; l < levels; ++l) {
        const uint32_t d = v % 3u;
        v /= 3u;
        h |= (uint32_t)(d == 1u) << l;
        m |= (uint32_t)(d == 2u) << l;
    }
    *hi = h;
    *mid = m;
}

// Lane task k (0 .. 15) of a sub-product: two t-blocks (16 output planes
// each) whose tiles add up to 17 for every k: k < 8 takes t-blocks k and
// 15 - k, k >= 8 takes 16 + (k - 8) and 31 - (k - 8).  Tile r (0 .. 16) is
// (t-block tbA, x-block jbA0 + r) for r < nA, else (tbB, jbB0 + r - nA).
struct BskTask {
    uint32_t tbA, tbB, nA, jbA0, jbB0;
};
QEXT_HD inline uint32_t bsk_jb_lo(uint32_t tb) { return tb > 16u ? tb - 16u : 0u; }
QEXT_HD inline uint32_t bsk_tiles(uint32_t tb) {
    const uint32_t hi = tb < 15u ? tb : 15u;
    return hi - bsk_jb_lo(tb) + 1u;
}
QEXT_HD inline BskTask bsk_task(uint32_t k) {
    BskTask t;
    if (k < 8u) {
        t.tbA = k;
        t.tbB = 15u - k;
    } else {
        t.tbA = 16u + (k - 8u);
        t.tbB = 31u - (k - 8u);
    }
    t.nA = bsk_tiles(t.tbA);
    t.jbA0 = bsk_jb_lo(t.tbA);
    t.jbB0 = bsk_jb_lo(t.tbB);
    return t;
}

// Launch geometry of (q, n_e), computed on the host and passed by value.
// LDS word offsets: the two plane arrays (bsk_pad layout, 265 q/256 words
// each), the materialized operands ("leaves") of the sub-products whose
// operand is a sum of segments (265 words each, per side), a zero block of
// 16 planes; the raw staging area ([side][word w][33]) aliases the leaves,
// and after the products the unreduced sum C (2q planes, plain) and the
// reduced planes Z (bsk_pad layout) alias everything.
struct BskGeom {
    uint32_t q, levels, np, n_leaf, qw, units;  // units: 16-byte loads per pair per side
    uint32_t pa;                 // words per plane array (265 q/256)
    uint32_t xpl, ypl;           // plane arrays
    uint32_t xlf, ylf;           // leaf arrays
    uint32_t raw;                // raw staging (aliases the leaves)
    uint32_t zero;               // 16 zero words
    uint32_t cs, zs;             // C and Z (after the products)
    uint32_t total;              // LDS words
    uint32_t threads, tasks;     // work-group size, lane tasks (16 np)
    uint32_t leaf_p[kBskMaxNp];  // sub-product of leaf li
    uint32_t xbase[kBskMaxNp];   // LDS word of plane 0 of sub-product p's X operand
    uint32_t ybase[kBskMaxNp];   // and of its Y operand
};

QEXT_HD inline uint32_t bsk_levels(uint32_t q) {
    return q == 512u ? 1u : q == 1024u ? 2u : q == 2048u ? 3u : 0u;
}

// false if q is not 512, 1024 or 2048.
inline bool bsk_geom(uint32_t q, BskGeom* g) {
    const uint32_t L = bsk_levels(q);
    if (!L) return false;
    BskGeom r{};
    r.q = q;
    r.levels = L;
    r.np = L == 1 ? 3u : L == 2 ? 9u : 27u;
    r.qw = q / 32;
    r.units = q / 128;
    r.pa = kBskLeaf * (q / kBskBase);
    r.xpl = 0;
    r.ypl = r.pa;
    r.xlf = 2 * r.pa;
    uint32_t n_leaf = 0;
    for (uint32_t p = 0; p < r.np; ++p) {
        uint32_t hi, mid;
        bsk_path(p, L, &hi, &mid);
        if (mid) r.leaf_p[n_leaf++] = p;
    }
    r.n_leaf = n_leaf;
    r.ylf = r.xlf + n_leaf * kBskLeaf;
    r.raw = r.xlf;
    const uint32_t leaves = 2 * n_leaf * kBskLeaf, raws = 2 * r.pa;
    r.zero = r.xlf + (leaves > raws ? leaves : raws);
    r.total = r.zero + 16;
    r.cs = 0;
    r.zs = 2 * q + (2 * q >> 8);  // C in cpad layout: plane c at c + c/256
    if (r.zs + r.pa > r.total) r.total = r.zs + r.pa;
    r.tasks = 16 * r.np;
    r.threads = (r.tasks + 63) / 64 * 64;
    if (r.threads < 256) r.threads = 256;
    for (uint32_t p = 0, li = 0; p < r.np; ++p) {
        uint32_t hi, mid;
        bsk_path(p, L, &hi, &mid);
        if (mid) {
            r.xbase[p] = r.xlf + kBskLeaf * li;
            r.ybase[p] = r.ylf + kBskLeaf * li;
            ++li;
        } else {  // a segment of the plane arrays: pad(256 hi + k) = 265 hi + pad(k)
            r.xbase[p] = r.xpl + kBskLeaf * hi;
            r.ybase[p] = r.ypl + kBskLeaf * hi;
        }
    }
    *g = r;
    return true;
}

}  // namespace qext
