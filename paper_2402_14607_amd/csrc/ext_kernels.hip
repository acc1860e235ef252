// ext_kernels.hip -- gfx950 kernels of the block-wise inner-product extractor.
//
// One block pair (x, y) of n bits each holds n_e elements of F_{2^q}; the
// output is Z = sum_i x_i * y_i in F_{2^q} (Def. 3.2), q bits per pair, for
// every pair of consecutive equal blocks (Algorithm 1).
//
// How it is computed (exact GF(2) arithmetic throughout):
//   * Field addition is XOR and reduction modulo P is linear, so the n_e
//     carry-less products x_i(t) y_i(t) are summed unreduced and the sum is
//     reduced once per pair.
//   * Each q x q carry-less product is split by L levels of Karatsuba into
//     3^L products of B = q / 2^L bits.  Karatsuba is linear in the
//     sub-products, so the sum over the n_e elements is taken in the split
//     domain: sub-product p of the pair is S_p = sum_i X_{i,p} Y_{i,p}, and
//     each S_p is scattered (XOR) into the unreduced result at its offsets.
//   * One lane computes one S_p with the shift-and-add (schoolbook) method on
//     32-bit words held in registers: for every bit s of every word of X,
//     acc ^= mask(bit) & (Y << s), the AND-XOR fused into one v_bitop3_b32.
//   * The 2q-1 bit sum is reduced modulo P = t^q + sum t^e + 1 (taps e < q/2)
//     in two folding passes, and the q-bit result is stored.
//
// Work decomposition: a work-group of 256 lanes owns `ppw` consecutive block
// pairs; its (pair, sub-product, element-group) items are spread over the
// lanes.  The pairs' input blocks are staged in LDS with coalesced loads
// (each input word is read from HBM once), every lane builds its Karatsuba
// operands from LDS, sub-products are combined with LDS atomic XOR, and the
// reduction reads the combined sum from LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ext_internal.h"

namespace qext {
namespace {

// acc ^= mask & y   (bitop3 truth table: src0 = 0xF0, src1 = 0xCC, src2 = 0xAA;
// (0xF0 & 0xCC) ^ 0xAA = 0x6A)
__device__ __forceinline__ uint32_t and_xor(uint32_t mask, uint32_t y, uint32_t acc) {
    return __builtin_amdgcn_bitop3_b32(mask, y, acc, 0x6A);
}

// all-ones if bit s of v is set, else zero
__device__ __forceinline__ uint32_t bit_mask(uint32_t v, uint32_t s) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)v, s, 1);
}

// ({hi, lo} >> sh) & 0xffffffff, sh in [0, 31]
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// acc[a + w] ^= mask(bit s of x[a]) & (y << s)[w]: one bit position s of
// every word of x, 0 < s < 32.
template <int BW>
__device__ __forceinline__ void clmul_shift(const uint32_t (&x)[BW], const uint32_t (&y)[BW],
                                            uint32_t (&acc)[2 * BW], uint32_t s) {
    uint32_t ys[BW + 1];
    ys[0] = y[0] << s;
#pragma unroll
    for (int w = 1; w < BW; ++w) ys[w] = funnel(y[w], y[w - 1], 32u - s);
    ys[BW] = y[BW - 1] >> (32u - s);
#pragma unroll
    for (int a = 0; a < BW; ++a) {
        const uint32_t m = bit_mask(x[a], s);
#pragma unroll
        for (int w = 0; w <= BW; ++w) acc[a + w] = and_xor(m, ys[w], acc[a + w]);
    }
}

// acc[0 .. 2BW) ^= x(t) * y(t) over GF(2), x and y BW words each.
template <int BW>
__device__ __forceinline__ void clmul_acc(const uint32_t (&x)[BW], const uint32_t (&y)[BW],
                                          uint32_t (&acc)[2 * BW]) {
    // shift 0: Y itself, word-aligned
#pragma unroll
    for (int a = 0; a < BW; ++a) {
        const uint32_t m = bit_mask(x[a], 0);
#pragma unroll
        for (int w = 0; w < BW; ++w) acc[a + w] = and_xor(m, y[w], acc[a + w]);
    }
    if constexpr (BW <= 4) {
        // short bodies: unrolled, so loop control does not take issue slots
#pragma unroll
        for (uint32_t s = 1; s < 32; ++s) clmul_shift<BW>(x, y, acc, s);
    } else {
#pragma unroll 1
        for (uint32_t s = 1; s < 32; ++s) clmul_shift<BW>(x, y, acc, s);
    }
}

// Read BW words from LDS (or global) at p into r (XOR-accumulate).
template <int BW>
__device__ __forceinline__ void xor_words(uint32_t (&r)[BW], const uint32_t* p) {
    if constexpr (BW % 4 == 0) {
        const uint4* p4 = reinterpret_cast<const uint4*>(p);
#pragma unroll
        for (int k = 0; k < BW / 4; ++k) {
            const uint4 v = p4[k];
            r[4 * k + 0] ^= v.x;
            r[4 * k + 1] ^= v.y;
            r[4 * k + 2] ^= v.z;
            r[4 * k + 3] ^= v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < BW; ++k) r[k] ^= p[k];
    }
}

// Karatsuba operand of one element: XOR of the B-bit segments hi_mask | sub
// for every subset sub of mid_mask (segment s = element bits [s*B, (s+1)*B)).
template <int BW>
__device__ __forceinline__ void form_operand(uint32_t (&r)[BW], const uint32_t* elem,
                                             uint32_t hi_mask, uint32_t mid_mask) {
#pragma unroll
    for (int w = 0; w < BW; ++w) r[w] = 0;
    uint32_t sub = mid_mask;
    for (;;) {
        xor_words<BW>(r, elem + (hi_mask | sub) * BW);
        if (sub == 0) break;
        sub = (sub - 1u) & mid_mask;
    }
}

// Karatsuba path of sub-product p: at each level it takes the low halves,
// the high halves or the sum of halves.  Bit l of a mask describes the level
// whose halves are B * 2^l bits (l = 0 is the lowest level).
//
// Outside kRankMin .. kRankMax levels p is read as base-3 digits, one per
// level (0 = low halves, 1 = high halves, 2 = sum of halves).  Within that
// range the 3^L paths are ranked by their number c of sum-of-halves levels,
// which sets the work of a lane outside its base product (2^c pieces per
// operand, 2^(L - c) scatter offsets): lanes of a wave holding neighbouring
// ranks then loop about equally often instead of as often as the wave's
// worst path.  The ranked masks come from a table built at compile time.
// MINL sets from how many levels a kernel ranks.  Unpadded shapes' whole-pair
// work-groups take their items rank-major (extract_group), so a wave holds a
// few neighbouring ranks, and rank from two levels on (paper block, three
// levels: 0.500 -> 0.463 ms per launch).  Padded shapes and slices take their
// items pair-major, so a wave spans every path of a pair unless L is large,
// and rank from five levels on (forward-block stress, six levels: -14 %); in
// the batched kernel only with bases of at most 8 words: at 16 words, where no
// shape reaches five levels, the variant that carried the ranking changed
// none of the loops' instruction counts and still measured 2-5 % slower.
constexpr uint32_t kRankMin = 2, kRankMax = 7;
constexpr uint32_t kRankedCount = 9 + 27 + 81 + 243 + 729 + 2187;  // 3^2 .. 3^7
struct RankedPaths {
    uint32_t v[kRankedCount];  // mid_mask << 16 | hi_mask
};
// Class c (C(L, c) 2^(L-c) paths) in the order of increasing c; within it
// the rank is comb * 2^(L-c) + bits: comb picks the sum-of-halves levels (the
// combinatorial number system), bits the low/high choice of the other levels,
// lowest level first, so that neighbouring ranks differ at low levels and the
// lanes' pieces and scatter offsets stay a few words apart (different LDS
// banks), as with the base-3 digits.
constexpr uint32_t choose(uint32_t n, uint32_t k) {
    if (k > n) return 0;
    uint32_t r = 1;
    for (uint32_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
constexpr RankedPaths make_ranked() {
    RankedPaths t{};
    uint32_t at = 0;
    for (uint32_t L = kRankMin; L <= kRankMax; ++L) {
        uint32_t n = 1;
        for (uint32_t i = 0; i < L; ++i) n *= 3;
        for (uint32_t p = 0; p < n; ++p) {
            uint32_t r = p, c = 0;
            for (;;) {
                const uint32_t cnt = choose(L, c) << (L - c);
                if (r < cnt) break;
                r -= cnt;
                ++c;
            }
            uint32_t bits = r & ((1u << (L - c)) - 1u), comb = r >> (L - c), k = c;
            uint32_t hm = 0, mm = 0;
            for (uint32_t pos = L; pos-- > 0;) {
                const uint32_t below = choose(pos, k);
                if (k > 0 && comb >= below) {
                    mm |= 1u << pos;
                    comb -= below;
                    --k;
                }
            }
            for (uint32_t pos = 0; pos < L; ++pos) {
                if (mm >> pos & 1u) continue;
                hm |= (bits & 1u) << pos;
                bits >>= 1;
            }
            t.v[at++] = mm << 16 | hm;
        }
    }
    return t;
}
__constant__ RankedPaths kRanked = make_ranked();

template <uint32_t MINL>
__device__ __forceinline__ void path_masks(uint32_t p, uint32_t levels, uint32_t& hi_mask,
                                           uint32_t& mid_mask) {
    if (levels >= MINL && levels >= kRankMin && levels <= kRankMax) {
        // table offset of L levels: 3^2 + ... + 3^(L-1) = (3^L - 9) / 2
        uint32_t p3 = 1;
        for (uint32_t l = 0; l < levels; ++l) p3 *= 3u;
        const uint32_t v = kRanked.v[(p3 - 9u) / 2u + p];
        hi_mask = v & 0xffffu;
        mid_mask = v >> 16;
        return;
    }
    uint32_t hm = 0, mm = 0, v = p;
    for (uint32_t l = 0; l < levels; ++l) {
        const uint32_t d = v % 3u;
        v /= 3u;
        hm |= (uint32_t)(d == 1u) << l;
        mm |= (uint32_t)(d == 2u) << l;
    }
    hi_mask = hm;
    mid_mask = mm;
}

// XOR a sub-product (2BW words) into the unreduced sum at cdst (LDS): a
// low-halves product lands at offsets {0, h}, a high-halves product at
// {h, 2h}, a sum-of-halves product at {h}, h = half size of that level; the
// offsets of all levels add up.
template <int BW>
__device__ __forceinline__ void scatter_acc(const uint32_t (&acc)[2 * BW], uint32_t hi_mask,
                                            uint32_t mid_mask, uint32_t lmask, uint32_t* cdst) {
    const uint32_t hm = hi_mask | mid_mask;
    const uint32_t lh = lmask & ~mid_mask;
    uint32_t sub = lh;
    for (;;) {
        const uint32_t off = BW * (hm + sub);
#pragma unroll
        for (int w = 0; w < 2 * BW; ++w) atomicXor(cdst + off + w, acc[w]);
        if (sub == 0) break;
        sub = (sub - 1u) & lh;
    }
}

// Reduce the npw unreduced sums at cs (2qw words each, complete and visible
// to the whole work-group) modulo P and store the q-bit results at out
// (qw words per pair); ds holds npw * dn words of scratch.  Ends after the
// last global store, without a barrier.
__device__ __forceinline__ void reduce_store(const ExtShape& sh, const uint32_t* cs,
                                             uint32_t cstride, uint32_t* ds,
                                             uint32_t* __restrict__ out, uint32_t npw) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = blockDim.x;
    const uint32_t qw = sh.qw, cw = 2 * qw;
    // ---- reduction modulo P ----------------------------------------------
    // C = C_lo + t^q C_hi with deg C_hi <= q-2, and t^q = 1 + sum_e t^e.
    // First pass: C_hi (1 + sum t^e); its part of degree >= q is
    // D = sum_e (C_hi >> (q - e)), of degree <= max_e - 2 < q/2, folded once more.
    const uint32_t dn = sh.dn;
    for (uint32_t i = tid; i < npw * dn; i += nt) {
        const uint32_t j = i / dn, k = i - j * dn;
        const uint32_t* hi = cs + j * cstride + qw;
        uint32_t d = 0;
        for (uint32_t t = 0; t < sh.n_taps; ++t) {
            const uint32_t r = sh.q - sh.taps[t];
            const uint32_t rw = r >> 5, rb = r & 31u;
            const uint32_t lo_i = k + rw, hi_i = k + rw + 1;
            const uint32_t lo = lo_i < qw ? hi[lo_i] : 0u;
            const uint32_t up = hi_i < qw ? hi[hi_i] : 0u;
            d ^= rb ? funnel(up, lo, rb) : lo;
        }
        ds[j * dn + k] = d;
    }
    __syncthreads();

    for (uint32_t i = tid; i < npw * qw; i += nt) {
        const uint32_t j = i / qw, w = i - j * qw;
        const uint32_t* c = cs + j * cstride;
        const uint32_t* hi = c + qw;
        const uint32_t* dd = ds + j * dn;
        uint32_t z = c[w] ^ hi[w] ^ (w < dn ? dd[w] : 0u);
        for (uint32_t t = 0; t < sh.n_taps; ++t) {
            const uint32_t e = sh.taps[t];
            const int32_t src = (int32_t)w - (int32_t)(e >> 5);
            const uint32_t eb = e & 31u;
            // word w of (C_hi << e)
            const uint32_t h1 = src >= 0 ? hi[src] : 0u;
            const uint32_t h0 = src >= 1 ? hi[src - 1] : 0u;
            z ^= eb ? funnel(h1, h0, 32u - eb) : h1;
            // word w of (D << e)
            const uint32_t d1 = (src >= 0 && (uint32_t)src < dn) ? dd[src] : 0u;
            const uint32_t d0 = (src >= 1 && (uint32_t)(src - 1) < dn) ? dd[src - 1] : 0u;
            z ^= eb ? funnel(d1, d0, 32u - eb) : d1;
        }
        out[(uint64_t)j * qw + w] = z;
    }
}

// 16 bytes [16k - lead, 16k - lead + 16) of the region [src, src + len)
// (lead = src & 15), zero outside it: one aligned 16-byte load when the chunk
// lies inside the region, single bytes otherwise, so no access leaves it.
__device__ __forceinline__ uint4 region_chunk(const uint8_t* __restrict__ src, uint32_t len,
                                              uint32_t lead, uint32_t k) {
    const uint32_t first = 16u * k;  // raw byte index of the chunk's first byte
    if (first >= lead && first + 16u <= lead + len)
        return reinterpret_cast<const uint4*>(src - lead)[k];
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    for (uint32_t b = 0; b < 16u; ++b) {
        const uint32_t rb = first + b;
        if (rb >= lead && rb < lead + len) v[b >> 2] |= (uint32_t)src[rb - lead] << (8u * (b & 3u));
    }
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// Padded layout of npw blocks in LDS for fields whose degree q is not a
// multiple of 32: element e of pair j occupies words [j*nw + e*qw, +qw), its
// q bits from the block's bytes [e*q/8, (e+1)*q/8) (blocks nbytes apart, no
// alignment assumed), zero above bit q.
//   1. Both sides' npw*nbytes bytes are copied as they are, X into the ys
//      area and Y into the xs area (raw byte lead + i = source byte i, lead =
//      src & 15), with 16-byte loads, all of a lane's loads in flight
//      together; each area has kPadSlack words of slack for the rounding.
//   2. Every lane gathers its slot words of both sides into registers with
//      funnel shifts; after a barrier it writes them to xs and ys.
// Ends with a barrier.
// (The element count, words and bytes per element and bytes per block come
// as scalars, so that a slice of a block -- n_e of its elements -- stages
// through the same code.)
__device__ __forceinline__ void stage_padded_core(uint32_t qw, uint32_t qb, uint32_t n_e,
                                                  uint32_t nbytes, const uint8_t* __restrict__ xb,
                                                  const uint8_t* __restrict__ yb, uint32_t* xs,
                                                  uint32_t* ys, uint32_t npw) {
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t nw = qw * n_e;
    const uint32_t len = npw * nbytes, total = npw * nw;
    const uint32_t lead_x = (uint32_t)((uintptr_t)xb & 15u), lead_y = (uint32_t)((uintptr_t)yb & 15u);
    const uint32_t nx = (lead_x + len + 15u) >> 4, ny = (lead_y + len + 15u) >> 4;
    uint32_t* raw_x = ys;  // X's raw bytes, in the ys area
    uint32_t* raw_y = xs;  // Y's raw bytes, in the xs area
    const uint32_t nc = nx > ny ? nx : ny;
#pragma unroll 4
    for (uint32_t k = tid; k < nc; k += nt) {
        const uint4 vx = region_chunk(xb, len, lead_x, k < nx ? k : 0);
        const uint4 vy = region_chunk(yb, len, lead_y, k < ny ? k : 0);
        if (k < nx) {
            raw_x[4 * k + 0] = vx.x;
            raw_x[4 * k + 1] = vx.y;
            raw_x[4 * k + 2] = vx.z;
            raw_x[4 * k + 3] = vx.w;
        }
        if (k < ny) {
            raw_y[4 * k + 0] = vy.x;
            raw_y[4 * k + 1] = vy.y;
            raw_y[4 * k + 2] = vy.z;
            raw_y[4 * k + 3] = vy.w;
        }
    }
    __syncthreads();
    // (pair, element, word) of slot word i = tid, and the step per nt words
    const uint32_t j0 = tid / nw, r0 = tid - j0 * nw, e0 = r0 / qw, w0 = r0 - e0 * qw;
    const uint32_t dj = nt / nw, rs = nt - dj * nw, de = rs / qw, dw = rs - de * qw;
    uint32_t hx[kPadRegs], hy[kPadRegs];
    uint32_t j = j0, e = e0, w = w0;
#pragma unroll
    for (uint32_t r = 0; r < kPadRegs; ++r) {
        if (tid + r * nt < total) {
            if (4u * w < qb) {
                const uint32_t o = j * nbytes + e * qb + 4u * w;  // byte in the region
                const uint32_t cnt = qb - 4u * w < 4u ? qb - 4u * w : 4u;  // >= 1
                const uint32_t keep = cnt < 4u ? (1u << (8u * cnt)) - 1u : ~0u;
                const uint32_t ox = o + lead_x, oy = o + lead_y;
                const uint32_t ax = ox >> 2, sx = (ox & 3u) * 8u, ay = oy >> 2, sy = (oy & 3u) * 8u;
                hx[r] = (sx ? funnel(raw_x[ax + 1], raw_x[ax], sx) : raw_x[ax]) & keep;
                hy[r] = (sy ? funnel(raw_y[ay + 1], raw_y[ay], sy) : raw_y[ay]) & keep;
            } else {  // a slot word above the element's bytes
                hx[r] = 0u;
                hy[r] = 0u;
            }
        }
        j += dj;
        e += de;
        w += dw;
        if (w >= qw) {
            w -= qw;
            e += 1;
        }
        if (e >= n_e) {
            e -= n_e;
            j += 1;
        }
    }
    __syncthreads();  // every read of the raw copies precedes every write
#pragma unroll
    for (uint32_t r = 0; r < kPadRegs; ++r) {
        const uint32_t i = tid + r * nt;
        if (i < total) {
            xs[i] = hx[r];
            ys[i] = hy[r];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void stage_padded(const ExtShape& sh, const uint8_t* __restrict__ xb,
                                             const uint8_t* __restrict__ yb, uint32_t* xs,
                                             uint32_t* ys, uint32_t npw) {
    stage_padded_core(sh.qw, sh.qbytes, sh.n_e, sh.nbytes, xb, yb, xs, ys, npw);
}

// reduce_store for padded shapes (q need not be a multiple of 32): C_hi = C >> q is first gathered
// into hs (qw words per pair) with funnel shifts, the folding passes are the
// same, the result is masked to q bits and stored as q/8 bytes per pair at
// outb (any alignment).  Ends after the last global store, without a barrier.
__device__ __forceinline__ void reduce_store_padded(const ExtShape& sh, const uint32_t* cs,
                                                    uint32_t* hs, uint32_t* ds,
                                                    uint8_t* __restrict__ outb, uint32_t npw) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = blockDim.x;
    const uint32_t qw = sh.qw, cw = 2 * qw, q0 = sh.q >> 5, r = sh.q & 31u;
    for (uint32_t i = tid; i < npw * qw; i += nt) {
        const uint32_t j = i / qw, w = i - j * qw;
        const uint32_t* c = cs + j * cw;
        hs[i] = funnel(c[q0 + w + 1], c[q0 + w], r);  // q0 + w + 1 <= 2qw - 1
    }
    __syncthreads();
    const uint32_t dn = sh.dn;
    for (uint32_t i = tid; i < npw * dn; i += nt) {
        const uint32_t j = i / dn, k = i - j * dn;
        const uint32_t* hi = hs + j * qw;
        uint32_t d = 0;
        for (uint32_t t = 0; t < sh.n_taps; ++t) {
            const uint32_t rr = sh.q - sh.taps[t];
            const uint32_t rw = rr >> 5, rb = rr & 31u;
            const uint32_t lo_i = k + rw, hi_i = k + rw + 1;
            const uint32_t lo = lo_i < qw ? hi[lo_i] : 0u;
            const uint32_t up = hi_i < qw ? hi[hi_i] : 0u;
            d ^= rb ? funnel(up, lo, rb) : lo;
        }
        ds[j * dn + k] = d;
    }
    __syncthreads();
    // words at or above bit q are not stored; the word holding bit q-1 is
    // masked to it
    const uint32_t q_words = (sh.q + 31u) >> 5;
    const uint32_t last_mask = r ? (1u << r) - 1u : ~0u;
    for (uint32_t i = tid; i < npw * qw; i += nt) {
        const uint32_t j = i / qw, w = i - j * qw;
        if (w >= q_words) continue;
        const uint32_t* hi = hs + j * qw;
        const uint32_t* dd = ds + j * dn;
        uint32_t z = cs[j * cw + w] ^ hi[w] ^ (w < dn ? dd[w] : 0u);
        for (uint32_t t = 0; t < sh.n_taps; ++t) {
            const uint32_t e = sh.taps[t];
            const int32_t src = (int32_t)w - (int32_t)(e >> 5);
            const uint32_t eb = e & 31u;
            const uint32_t h1 = src >= 0 ? hi[src] : 0u;
            const uint32_t h0 = src >= 1 ? hi[src - 1] : 0u;
            z ^= eb ? funnel(h1, h0, 32u - eb) : h1;
            const uint32_t d1 = (src >= 0 && (uint32_t)src < dn) ? dd[src] : 0u;
            const uint32_t d0 = (src >= 1 && (uint32_t)(src - 1) < dn) ? dd[src - 1] : 0u;
            z ^= eb ? funnel(d1, d0, 32u - eb) : d1;
        }
        if (w == q_words - 1) z &= last_mask;
        uint8_t* o = outb + (uint64_t)j * sh.qbytes + 4u * w;
        const uint32_t cnt = sh.qbytes - 4u * w < 4u ? sh.qbytes - 4u * w : 4u;
        for (uint32_t b = 0; b < cnt; ++b) o[b] = (uint8_t)(z >> (8u * b));
    }
}

// One work-group's share: npw consecutive block pairs of one stream with
// shape sh (npw <= sh.ppw); xb, yb point at the first pair's blocks and outb
// at its output (bytes; 4-byte aligned unless the shape is padded).  lds
// holds sh.lds_words words, plus group_pad_words(sh) with RMAJOR.  Ends after
// the last global store, without a barrier.
//
// Items are (pair, sub-product, element group).  RMAJOR takes them rank-major
// (lanes next to each other hold the same sub-product of different pairs), so
// that with the ranked order the lanes of a wave share their number of
// sum-of-halves levels and loop equally often; the staged blocks and the sums
// then sit at padded per-pair strides (blocks + 4 words, sums + 1) so that the
// pairs' words fall in different LDS banks.  Otherwise items are pair-major.
template <int BW, bool PAD, uint32_t MINL, bool RMAJOR>
__device__ __forceinline__ void extract_group(const ExtShape& sh, const uint8_t* __restrict__ xb,
                                              const uint8_t* __restrict__ yb,
                                              uint8_t* __restrict__ outb, uint32_t npw,
                                              uint32_t* lds) {
    static_assert(!(PAD && RMAJOR), "padded shapes keep their own staging layout");
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = blockDim.x;  // sh.threads lanes
    const uint32_t nw = sh.nw, qw = sh.qw, cw = 2 * qw;
    const uint32_t nws = RMAJOR ? nw + 4u : nw;  // staged words per pair
    const uint32_t cws = RMAJOR ? cw + 1u : cw;  // sum words per pair
    const uint32_t* xg = reinterpret_cast<const uint32_t*>(xb);
    const uint32_t* yg = reinterpret_cast<const uint32_t*>(yb);
    // padded shapes: kPadSlack words after each staged area (raw copies)
    const uint32_t area = (sh.stage ? sh.ppw * nws : 0) + (PAD ? kPadSlack : 0);
    uint32_t* xs = lds;                               // [ppw][nws]  (staged X)
    uint32_t* ys = xs + area;                         // [ppw][nws]  (staged Y)
    uint32_t* cs = ys + area;                         // [ppw][cws]  unreduced sums
    uint32_t* ds = cs + sh.ppw * cws;                 // [ppw][dn]   second-pass words
    uint32_t* hs = ds + sh.ppw * sh.dn;               // [ppw][qw]   C >> q (padded shapes)

    for (uint32_t i = tid; i < npw * cws; i += nt) cs[i] = 0;
    if constexpr (PAD) {
        stage_padded(sh, xb, yb, xs, ys, npw);  // padded shapes are always staged
    } else if (sh.stage) {
        if constexpr (RMAJOR) {
            for (uint32_t j = 0; j < npw; ++j)
                for (uint32_t k = tid; k < nw; k += nt) {
                    xs[j * nws + k] = xg[j * nw + k];
                    ys[j * nws + k] = yg[j * nw + k];
                }
        } else {
            for (uint32_t i = tid; i < npw * nw; i += nt) {
                xs[i] = xg[i];
                ys[i] = yg[i];
            }
        }
    }
    __syncthreads();

    // ---- sub-products ---------------------------------------------------
    const uint32_t per_pair = sh.np * sh.groups;
    const uint32_t per_rank = npw * sh.groups;
    const uint32_t items = npw * per_pair;
    const uint32_t lmask = (1u << sh.levels) - 1u;
    for (uint32_t it = tid; it < items; it += nt) {
        uint32_t j, p, g;
        if constexpr (RMAJOR) {
            p = it / per_rank;
            const uint32_t rem = it - p * per_rank;
            j = rem / sh.groups;
            g = rem - j * sh.groups;
        } else {
            j = it / per_pair;
            const uint32_t rem = it - j * per_pair;
            p = rem / sh.groups;
            g = rem - p * sh.groups;
        }
        uint32_t hi_mask, mid_mask;
        path_masks<MINL>(p, sh.levels, hi_mask, mid_mask);
        uint32_t acc[2 * BW];
#pragma unroll
        for (int w = 0; w < 2 * BW; ++w) acc[w] = 0;

        // elements of group g (the last group may hold fewer)
        const uint32_t e_end = (g + 1) * sh.epg < sh.n_e ? (g + 1) * sh.epg : sh.n_e;
        for (uint32_t e = g * sh.epg; e < e_end; ++e) {
            uint32_t xo[BW], yo[BW];
            if (sh.stage) {  // operands from the LDS copy
                form_operand<BW>(xo, xs + j * nws + e * qw, hi_mask, mid_mask);
                form_operand<BW>(yo, ys + j * nws + e * qw, hi_mask, mid_mask);
            } else {         // straight from HBM (one sub-product per element)
                form_operand<BW>(xo, xg + (uint64_t)j * nw + e * qw, hi_mask, mid_mask);
                form_operand<BW>(yo, yg + (uint64_t)j * nw + e * qw, hi_mask, mid_mask);
            }
            clmul_acc<BW>(xo, yo, acc);
        }

        scatter_acc<BW>(acc, hi_mask, mid_mask, lmask, cs + j * cws);
    }
    __syncthreads();
    if constexpr (PAD)
        reduce_store_padded(sh, cs, hs, ds, outb, npw);
    else
        reduce_store(sh, cs, cws, ds, reinterpret_cast<uint32_t*>(outb), npw);
}

// One slice of one block pair, for pairs with more sub-products than a
// work-group has lanes: items [item0, item0 + n_items) of the pair's
// n_e * 3^L (element, sub-product) items in element-major order, one base
// product each.  The slice's part of the unreduced sum (2qw words, the other
// slices' parts XOR to the rest) is stored at part; combine_kernel adds the
// parts and reduces.  Only the elements the slice touches are staged.  Ends
// after the last global store, without a barrier.
template <int BW, uint32_t MINL>
__device__ __forceinline__ void extract_slice(const ExtShape& sh, const uint32_t* __restrict__ xg,
                                              const uint32_t* __restrict__ yg,
                                              uint32_t* __restrict__ part, uint32_t item0,
                                              uint32_t n_items, uint32_t* lds) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = blockDim.x;
    const uint32_t qw = sh.qw, cw = 2 * qw;
    const uint32_t e0 = item0 / sh.np;
    const uint32_t sw = ((item0 + n_items - 1) / sh.np - e0 + 1) * qw;  // staged words per side
    uint32_t* xs = lds;                          // [sw] (staged X elements)
    uint32_t* ys = xs + (sh.stage ? sw : 0);     // [sw] (staged Y elements)
    uint32_t* cs = ys + (sh.stage ? sw : 0);     // [2qw] partial unreduced sum

    for (uint32_t i = tid; i < cw; i += nt) cs[i] = 0;
    if (sh.stage) {
        for (uint32_t i = tid; i < sw; i += nt) {
            xs[i] = xg[e0 * qw + i];
            ys[i] = yg[e0 * qw + i];
        }
    }
    __syncthreads();

    const uint32_t lmask = (1u << sh.levels) - 1u;
    for (uint32_t it = tid; it < n_items; it += nt) {
        const uint32_t gi = item0 + it;
        const uint32_t e = gi / sh.np;
        const uint32_t p = gi - e * sh.np;
        uint32_t hi_mask, mid_mask;
        path_masks<MINL>(p, sh.levels, hi_mask, mid_mask);
        uint32_t acc[2 * BW];
#pragma unroll
        for (int w = 0; w < 2 * BW; ++w) acc[w] = 0;
        uint32_t xo[BW], yo[BW];
        if (sh.stage) {
            form_operand<BW>(xo, xs + (e - e0) * qw, hi_mask, mid_mask);
            form_operand<BW>(yo, ys + (e - e0) * qw, hi_mask, mid_mask);
        } else {
            form_operand<BW>(xo, xg + e * qw, hi_mask, mid_mask);
            form_operand<BW>(yo, yg + e * qw, hi_mask, mid_mask);
        }
        clmul_acc<BW>(xo, yo, acc);
        scatter_acc<BW>(acc, hi_mask, mid_mask, lmask, cs);
    }
    __syncthreads();
    for (uint32_t i = tid; i < cw; i += nt) part[i] = cs[i];
}

// One slice of one block pair of a padded shape, for blocks too large for
// one work-group: elements [e0, e0 + ne) (block bytes [e0 q/8, (e0 + ne) q/8),
// any alignment), every sub-product of each.  They are staged in the padded
// layout (2 (ne qw + kPadSlack) words of LDS), the slice's part of the
// unreduced sum (2qw words, the other slices' parts XOR to the rest) is
// stored at part, and combine_padded_kernel adds the parts, reduces and
// stores the pair.  Ends after the last global store, without a barrier.
template <int BW, uint32_t MINL>
__device__ __forceinline__ void extract_slice_padded(const ExtShape& sh,
                                                     const uint8_t* __restrict__ xb,
                                                     const uint8_t* __restrict__ yb,
                                                     uint32_t* __restrict__ part, uint32_t e0,
                                                     uint32_t ne, uint32_t* lds) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nt = blockDim.x;
    const uint32_t qw = sh.qw, cw = 2 * qw, qb = sh.qbytes;
    const uint32_t area = ne * qw + kPadSlack;
    uint32_t* xs = lds;        // [ne][qw] (staged X elements)
    uint32_t* ys = xs + area;  // [ne][qw] (staged Y elements)
    uint32_t* cs = ys + area;  // [2qw] partial unreduced sum

    for (uint32_t i = tid; i < cw; i += nt) cs[i] = 0;
    stage_padded_core(qw, qb, ne, ne * qb, xb + (uint64_t)e0 * qb, yb + (uint64_t)e0 * qb, xs,
                      ys, 1);  // ends with a barrier

    const uint32_t lmask = (1u << sh.levels) - 1u;
    const uint32_t n_items = ne * sh.np;
    for (uint32_t it = tid; it < n_items; it += nt) {
        const uint32_t e = it / sh.np;
        const uint32_t p = it - e * sh.np;
        uint32_t hi_mask, mid_mask;
        path_masks<MINL>(p, sh.levels, hi_mask, mid_mask);
        uint32_t acc[2 * BW];
#pragma unroll
        for (int w = 0; w < 2 * BW; ++w) acc[w] = 0;
        uint32_t xo[BW], yo[BW];
        form_operand<BW>(xo, xs + e * qw, hi_mask, mid_mask);
        form_operand<BW>(yo, ys + e * qw, hi_mask, mid_mask);
        clmul_acc<BW>(xo, yo, acc);
        scatter_acc<BW>(acc, hi_mask, mid_mask, lmask, cs);
    }
    __syncthreads();
    for (uint32_t i = tid; i < cw; i += nt) part[i] = cs[i];
}

// Plain form: work-group g takes pairs [g*ppw, (g+1)*ppw) of one stream.
// PAD: the shape is padded (q not a multiple of 32).
template <int BW, bool PAD>
__global__ void __launch_bounds__(kMaxThreads)
ext_ip_kernel(const uint8_t* __restrict__ x, const uint8_t* __restrict__ y,
              uint8_t* __restrict__ out, uint64_t n_pairs, ExtShape sh) {
    extern __shared__ uint32_t lds[];
    const uint64_t pair0 = (uint64_t)blockIdx.x * sh.ppw;
    if (pair0 >= n_pairs) return;
    const uint64_t left = n_pairs - pair0;
    const uint32_t npw = left < sh.ppw ? (uint32_t)left : sh.ppw;
    extract_group<BW, PAD, PAD ? 5u : 2u, !PAD>(sh, x + pair0 * sh.nbytes, y + pair0 * sh.nbytes,
                                                out + pair0 * sh.qbytes, npw, lds);
}

// From how many levels the batched kernel of base size BW ranks the
// sub-products of its slices and padded tiles (items pair-major): only bases
// of at most 8 words reach five or more levels in practice.  Unpadded whole
// tiles go rank-major, as in the plain kernel.
template <int BW>
constexpr uint32_t kBatchRank = BW <= 8 ? 5u : 100u;

// Batched form: a persistent grid drains a device work queue of tiles
// (stream, first pair, pair count; or one slice of one pair) shared by many
// streams of different shapes.  Each work-group takes the next tile with one atomic add on the
// queue head and stops once the head passes n_tiles, so every wave exits.
// PAD: every stream of the launch has a padded shape (slices of a padded
// shape are element ranges).
template <int BW, bool PAD>
__global__ void __launch_bounds__(kMaxThreads)
ext_batch_kernel(const BatchStream* __restrict__ streams, const BatchTile* __restrict__ tiles,
                 uint32_t n_tiles, uint32_t* __restrict__ head, uint32_t* __restrict__ part) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(head, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(next);
        if (t >= n_tiles) break;
        const BatchTile tile = tiles[t];
        const BatchStream& st = streams[tile.stream];
        const ExtShape& sh = st.shape;  // read in place (a local copy would go to scratch)
        const uint8_t* xb = st.x + tile.in_pair0 * sh.nbytes;
        const uint8_t* yb = st.y + tile.in_pair0 * sh.nbytes;
        if (tile.n_items) {  // one slice of one pair; out_off is its part's word offset
            if constexpr (PAD)  // elements [item0, item0 + n_items)
                extract_slice_padded<BW, kBatchRank<BW>>(sh, xb, yb, part + tile.out_off,
                                                         tile.item0, tile.n_items, lds);
            else  // items [item0, item0 + n_items)
                extract_slice<BW, kBatchRank<BW>>(sh, reinterpret_cast<const uint32_t*>(xb),
                                  reinterpret_cast<const uint32_t*>(yb), part + tile.out_off,
                                  tile.item0, tile.n_items, lds);
        } else
            extract_group<BW, PAD, PAD ? kBatchRank<BW> : 2u, !PAD>(
                sh, xb, yb, st.out + tile.out_off, tile.npw, lds);
        __syncthreads();  // LDS and `next` are reused by the next tile
    }
}

// Served cycles with sliced pairs: work-group b takes jobs b, b + grid, ...;
// a job XORs the n_parts consecutive parts (2qw words each) of one pair,
// reduces the sum modulo P and stores the pair's output.  lds holds
// 2qw + dn words of the largest shape among the jobs.
__global__ void __launch_bounds__(kThreads)
combine_kernel(const BatchStream* __restrict__ streams, const CombineJob* __restrict__ jobs,
               uint32_t n_jobs, const uint32_t* __restrict__ part) {
    extern __shared__ uint32_t lds[];
    for (uint32_t jb = blockIdx.x; jb < n_jobs; jb += gridDim.x) {
        const CombineJob job = jobs[jb];
        const BatchStream& st = streams[job.stream];
        const ExtShape& sh = st.shape;
        const uint32_t cw = 2 * sh.qw;
        const uint32_t* src = part + job.part_word0;
        if ((cw & 3u) == 0 && (job.part_word0 & 3u) == 0) {
            // 16-byte loads, four parts' loads in flight before they are used
            const uint4* s4 = reinterpret_cast<const uint4*>(src);
            const uint32_t c4 = cw / 4;
            for (uint32_t i = threadIdx.x; i < c4; i += blockDim.x) {
                uint4 v = s4[i];
                uint32_t k = 1;
                for (; k + 4 <= job.n_parts; k += 4) {
                    const uint4 a = s4[(uint64_t)k * c4 + i];
                    const uint4 b = s4[(uint64_t)(k + 1) * c4 + i];
                    const uint4 c = s4[(uint64_t)(k + 2) * c4 + i];
                    const uint4 d = s4[(uint64_t)(k + 3) * c4 + i];
                    v.x ^= a.x ^ b.x ^ c.x ^ d.x;
                    v.y ^= a.y ^ b.y ^ c.y ^ d.y;
                    v.z ^= a.z ^ b.z ^ c.z ^ d.z;
                    v.w ^= a.w ^ b.w ^ c.w ^ d.w;
                }
                for (; k < job.n_parts; ++k) {
                    const uint4 a = s4[(uint64_t)k * c4 + i];
                    v.x ^= a.x;
                    v.y ^= a.y;
                    v.z ^= a.z;
                    v.w ^= a.w;
                }
                lds[4 * i + 0] = v.x;
                lds[4 * i + 1] = v.y;
                lds[4 * i + 2] = v.z;
                lds[4 * i + 3] = v.w;
            }
        } else {
            for (uint32_t i = threadIdx.x; i < cw; i += blockDim.x) {
                uint32_t v = 0;
                for (uint32_t k = 0; k < job.n_parts; ++k) v ^= src[(uint64_t)k * cw + i];
                lds[i] = v;
            }
        }
        __syncthreads();
        reduce_store(sh, lds, cw, lds + cw, reinterpret_cast<uint32_t*>(st.out + job.out_byte0), 1);
        __syncthreads();  // lds is reused by the next job
    }
}

// Padded shapes' sliced pairs: as combine_kernel, with the reduction and the
// byte-granular store of padded shapes.  Job outputs may start at any byte
// (out_byte0).  lds holds 3qw + dn words of the largest shape among the jobs.
__global__ void __launch_bounds__(kThreads)
combine_padded_kernel(const BatchStream* __restrict__ streams, const CombineJob* __restrict__ jobs,
                      uint32_t n_jobs, const uint32_t* __restrict__ part) {
    extern __shared__ uint32_t lds[];
    for (uint32_t jb = blockIdx.x; jb < n_jobs; jb += gridDim.x) {
        const CombineJob job = jobs[jb];
        const BatchStream& st = streams[job.stream];
        const ExtShape& sh = st.shape;
        const uint32_t cw = 2 * sh.qw;
        const uint32_t* src = part + job.part_word0;
        for (uint32_t i = threadIdx.x; i < cw; i += blockDim.x) {
            // eight parts' loads in flight before they are used (the parts
            // were just written by other CUs: every load goes past this L2)
            uint32_t v = 0, k = 0;
            for (; k + 8 <= job.n_parts; k += 8) {
                uint32_t a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = src[(uint64_t)(k + u) * cw + i];
#pragma unroll
                for (int u = 0; u < 8; ++u) v ^= a[u];
            }
            for (; k < job.n_parts; ++k) v ^= src[(uint64_t)k * cw + i];
            lds[i] = v;
        }
        __syncthreads();
        reduce_store_padded(sh, lds, lds + cw, lds + cw + sh.qw, st.out + job.out_byte0, 1);
        __syncthreads();  // lds is reused by the next job
    }
}

// Start of a served cycle, reading the host's pinned staging area directly:
// every work-group copies its share of the descriptors' byte ranges into the
// channels' rings (16-byte accesses when aligned), the grid copies the cycle's
// metadata (stream table and tiles) into device memory, and work-group 0 clears
// the queue heads.  No copy engine is involved, so the cycle's kernels follow
// one another on one stream with no host-side dependency.
__global__ void __launch_bounds__(kThreads)
stage_kernel(const uint8_t* __restrict__ src, const ScatterDesc* __restrict__ descs,
             uint32_t n_descs, const uint4* __restrict__ meta_src, uint4* __restrict__ meta_dst,
             uint32_t meta_vec, uint32_t* __restrict__ heads, uint32_t n_heads) {
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < n_heads; i += kThreads) heads[i] = 0u;
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < meta_vec; i += gridDim.x * kThreads)
        meta_dst[i] = meta_src[i];
    for (uint32_t d = blockIdx.x; d < n_descs; d += gridDim.x) {
        const ScatterDesc sd = descs[d];
        const uint8_t* s = src + sd.src_off;
        uint8_t* t = sd.dst;
        if ((((uintptr_t)s | (uintptr_t)t | sd.len) & 15u) == 0) {
            // four 16-byte loads in flight per lane before their stores (a
            // 16 KiB piece is one round trip over the bus)
            const uint4* s16 = reinterpret_cast<const uint4*>(s);
            uint4* t16 = reinterpret_cast<uint4*>(t);
            const uint32_t n16 = sd.len / 16;
            uint32_t i = threadIdx.x;
            for (; i + 3 * kThreads < n16; i += 4 * kThreads) {
                const uint4 a = s16[i];
                const uint4 b = s16[i + kThreads];
                const uint4 c = s16[i + 2 * kThreads];
                const uint4 d = s16[i + 3 * kThreads];
                t16[i] = a;
                t16[i + kThreads] = b;
                t16[i + 2 * kThreads] = c;
                t16[i + 3 * kThreads] = d;
            }
            for (; i < n16; i += kThreads) t16[i] = s16[i];
        } else if ((((uintptr_t)s | (uintptr_t)t | sd.len) & 3u) == 0) {
            const uint32_t* s4 = reinterpret_cast<const uint32_t*>(s);
            uint32_t* t4 = reinterpret_cast<uint32_t*>(t);
            for (uint32_t i = threadIdx.x; i < sd.len / 4; i += kThreads) t4[i] = s4[i];
        } else {
            for (uint32_t i = threadIdx.x; i < sd.len; i += kThreads) t[i] = s[i];
        }
    }
}

// Issue-rate probe: every lane runs eight independent v_bitop3_b32 chains
// (the extraction kernel's AND-XOR) plus one funnel shift per round of eight,
// and writes one word, out[global id], so the work cannot be dropped.
__global__ void __launch_bounds__(kThreads)
valu_probe_kernel(uint32_t* __restrict__ out, uint32_t seed, uint32_t iters) {
    const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
    uint32_t a[8], m = seed * gid + 0x9e3779b9u;
    const uint32_t y = gid ^ 0x5bd1e995u;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = gid + (uint32_t)j;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = and_xor(m, y + (uint32_t)j, a[j]);
            m = funnel(m, y, 1u);
        }
    }
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) v ^= a[j];
    out[gid] = v;
}

// Clears the queue head (a kernel, not a memset node, so that the pair can be
// captured in a graph and replayed).
__global__ void reset_head_kernel(uint32_t* head) {
    if (threadIdx.x == 0) *head = 0u;
}

template <int BW>
hipError_t launch_bw(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                     uint64_t n_pairs, hipStream_t stream) {
    const uint64_t groups = (n_pairs + s.ppw - 1) / s.ppw;
    if (groups > 0x7fffffffull) return hipErrorInvalidValue;
    if (s.padded)
        hipLaunchKernelGGL((ext_ip_kernel<BW, true>), dim3((uint32_t)groups), dim3(s.threads),
                           group_lds_bytes(s), stream, x, y, out, n_pairs, s);
    else
        hipLaunchKernelGGL((ext_ip_kernel<BW, false>), dim3((uint32_t)groups), dim3(s.threads),
                           group_lds_bytes(s), stream, x, y, out, n_pairs, s);
    return hipGetLastError();
}

template <int BW>
hipError_t launch_batch_only_bw(uint32_t threads, bool padded, const BatchStream* streams,
                                const BatchTile* tiles, uint32_t n_tiles, uint32_t* head,
                                uint32_t* part, uint32_t grid, uint32_t lds_bytes,
                                hipStream_t stream) {
    if (padded)
        hipLaunchKernelGGL((ext_batch_kernel<BW, true>), dim3(grid), dim3(threads), lds_bytes,
                           stream, streams, tiles, n_tiles, head, part);
    else
        hipLaunchKernelGGL((ext_batch_kernel<BW, false>), dim3(grid), dim3(threads), lds_bytes,
                           stream, streams, tiles, n_tiles, head, part);
    return hipGetLastError();
}

template <int BW>
hipError_t launch_batch_bw(uint32_t threads, bool padded, const BatchStream* streams,
                           const BatchTile* tiles, uint32_t n_tiles, uint32_t* head, uint32_t grid,
                           uint32_t lds_bytes, hipStream_t stream) {
    hipLaunchKernelGGL(reset_head_kernel, dim3(1), dim3(64), 0, stream, head);
    return launch_batch_only_bw<BW>(threads, padded, streams, tiles, n_tiles, head,
                                    static_cast<uint32_t*>(nullptr), grid, lds_bytes, stream);
}

template <int BW>
hipError_t occupancy_bw(uint32_t threads, bool padded, uint32_t lds_bytes, int* blocks_per_cu) {
    if (padded)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            blocks_per_cu, ext_batch_kernel<BW, true>, threads, lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, ext_batch_kernel<BW, false>,
                                                        threads, lds_bytes);
}

}  // namespace

#define QEXT_BW_CASES(F, ...)                      \
    switch (bw) {                                  \
        case 1: return F<1>(__VA_ARGS__);          \
        case 2: return F<2>(__VA_ARGS__);          \
        case 3: return F<3>(__VA_ARGS__);          \
        case 4: return F<4>(__VA_ARGS__);          \
        case 5: return F<5>(__VA_ARGS__);          \
        case 6: return F<6>(__VA_ARGS__);          \
        case 7: return F<7>(__VA_ARGS__);          \
        case 8: return F<8>(__VA_ARGS__);          \
        case 9: return F<9>(__VA_ARGS__);          \
        case 11: return F<11>(__VA_ARGS__);        \
        case 13: return F<13>(__VA_ARGS__);        \
        case 15: return F<15>(__VA_ARGS__);        \
        case 16: return F<16>(__VA_ARGS__);        \
        default: return hipErrorInvalidValue;      \
    }

hipError_t launch_batch(uint32_t bw, uint32_t threads, bool padded, const BatchStream* streams,
                        const BatchTile* tiles, uint32_t n_tiles, uint32_t* head, uint32_t grid,
                        uint32_t lds_bytes, hipStream_t stream) {
    if (n_tiles == 0) return hipSuccess;
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64) return hipErrorInvalidValue;
    QEXT_BW_CASES(launch_batch_bw, threads, padded, streams, tiles, n_tiles, head, grid, lds_bytes,
                  stream)
}

hipError_t launch_stage(const uint8_t* src, const ScatterDesc* descs, uint32_t n_descs,
                        const void* meta_src, void* meta_dst, uint32_t meta_bytes, uint32_t* heads,
                        uint32_t n_heads, hipStream_t stream) {
    if (meta_bytes % 16) return hipErrorInvalidValue;
    const uint32_t meta_vec = meta_bytes / 16;
    uint32_t grid = n_descs;
    grid = grid > (meta_vec + kThreads - 1) / kThreads ? grid : (meta_vec + kThreads - 1) / kThreads;
    grid = grid < 1u ? 1u : (grid > 8192u ? 8192u : grid);
    hipLaunchKernelGGL(stage_kernel, dim3(grid), dim3(kThreads), 0, stream, src, descs, n_descs,
                       static_cast<const uint4*>(meta_src), static_cast<uint4*>(meta_dst), meta_vec,
                       heads, n_heads);
    return hipGetLastError();
}

hipError_t launch_batch_noreset(uint32_t bw, uint32_t threads, bool padded,
                                const BatchStream* streams, const BatchTile* tiles,
                                uint32_t n_tiles, uint32_t* head, uint32_t* part, uint32_t grid,
                                uint32_t lds_bytes, hipStream_t stream) {
    if (n_tiles == 0) return hipSuccess;
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64) return hipErrorInvalidValue;
    QEXT_BW_CASES(launch_batch_only_bw, threads, padded, streams, tiles, n_tiles, head, part, grid,
                  lds_bytes, stream)
}

hipError_t launch_combine(const BatchStream* streams, const CombineJob* jobs, uint32_t n_jobs,
                          const uint32_t* part, uint32_t grid, uint32_t lds_bytes,
                          hipStream_t stream) {
    if (n_jobs == 0) return hipSuccess;
    if (grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(combine_kernel, dim3(grid), dim3(kThreads), lds_bytes, stream, streams, jobs,
                       n_jobs, part);
    return hipGetLastError();
}

hipError_t launch_combine_padded(const BatchStream* streams, const CombineJob* jobs,
                                 uint32_t n_jobs, const uint32_t* part, uint32_t grid,
                                 uint32_t lds_bytes, hipStream_t stream) {
    if (n_jobs == 0) return hipSuccess;
    if (grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(combine_padded_kernel, dim3(grid), dim3(kThreads), lds_bytes, stream,
                       streams, jobs, n_jobs, part);
    return hipGetLastError();
}

hipError_t launch_valu_probe(uint32_t* out, uint32_t blocks, uint32_t iters, hipStream_t stream) {
    if (!out || blocks == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kThreads), 0, stream, out, 7u, iters);
    return hipGetLastError();
}

hipError_t batch_occupancy(uint32_t bw, uint32_t threads, bool padded, uint32_t lds_bytes,
                           int* blocks_per_cu) {
    QEXT_BW_CASES(occupancy_bw, threads, padded, lds_bytes, blocks_per_cu)
}

hipError_t launch_extract(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                          uint64_t n_pairs, hipStream_t stream) {
    if (n_pairs == 0) return hipSuccess;
    if (s.threads == 0 || s.threads > (uint32_t)kMaxThreads || s.threads % 64)
        return hipErrorInvalidValue;
    const uint32_t bw = s.bw;
    QEXT_BW_CASES(launch_bw, s, x, y, out, n_pairs, stream)
}

}  // namespace qext
