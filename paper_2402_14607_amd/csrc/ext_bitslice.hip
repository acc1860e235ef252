// ext_bitslice.hip -- bit-sliced kernel for small fields (q <= 128) with many
// elements per block, such as the paper's own point (71 elements of F_2^80).
//
// A word-level product of q <= 128 bits spends most of its issue slots on
// shifts and masks (a 96-bit schoolbook product: 7 of 19).  Here a work-group
// takes 32 block pairs and transposes them so that bit p of a 32-bit "plane"
// word belongs to pair p: plane (e, j) holds bit j of element e of all 32
// pairs.  The carry-less product of every element pair is then
//     c[t] ^= x[j] & y[t - j]      (one v_bitop3_b32 per (j, t), 32 pairs at once)
// with no shift and no mask, summed over the elements as the paper's inner
// product (Def. 3.2) asks, reduced modulo P plane by plane, and transposed
// back into q-bit outputs.
//
// The 32 pairs' blocks are one contiguous region per side.  The elements are
// taken in chunks of ec; for each chunk a work-group (256 lanes)
//   1. stages the chunk's bytes of both sides in LDS as they are, with
//      16-byte loads (issued after the products of the chunk before, when
//      the raw area is free);
//   2. transposes them: item (side, word w, element) gathers word w of the
//      element of the 32 pairs, transposes the 32x32 bit matrix in registers
//      and writes 32 planes (zero at or above q); Y planes have zero margins
//      before (kYLo) and after (kYHi);
//   3. multiplies: lane (16x16 tile position (j-block, t-block offset),
//      element subset) accumulates the tile's output planes in registers
//      (x[j] for 16 j, y[t - j] from two windows of 16 and 15 planes) over
//      its elements of the chunk, keeping the sums across chunks.
// After the last chunk the lanes XOR their sums into the shared sum C (LDS
// atomics); then C is reduced modulo P, one output plane per lane (two
// folding passes, taps at most q/2); lane w transposes planes 32w .. 32w+31 back
// into word w of the 32 outputs, and the work-group stores its npw*q/8 bytes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ext_internal.h"

namespace qext {
namespace {

constexpr uint32_t kBsPairs = 32;   // pairs per work-group (bits of a plane)
constexpr uint32_t kTile = 16;      // planes per tile side
constexpr uint32_t kYLo = 16;       // zero Y planes before each element
constexpr uint32_t kYHi = 32;       // zero Y planes after each element's jp planes

__device__ __forceinline__ uint32_t bs_and_xor(uint32_t a, uint32_t b, uint32_t acc) {
    return __builtin_amdgcn_bitop3_b32(a, b, acc, 0x6A);  // (a & b) ^ acc
}

// One block-swap step of the 32x32 transpose: for rows r with bit J clear,
// the columns of row r with bit J set are exchanged with the columns of row
// r + J with bit J clear (M selects the columns with bit J clear).  Steps of
// 16 and 8 move whole bytes (one v_perm_b32 per row); the others take a
// shift and a bit select (v_bitop3_b32 0xD8: (a & ~m) | (b & m)) per row.
__device__ __forceinline__ uint32_t bs_select(uint32_t a, uint32_t b, uint32_t m) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0xD8);
}

template <int J, uint32_t M>
__device__ __forceinline__ void transpose_step(uint32_t (&a)[32]) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        if (r & J) continue;
        const uint32_t lo = a[r], hi = a[r + J];
        if constexpr (J == 16) {
            a[r] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);      // lo.b0 lo.b1 hi.b0 hi.b1
            a[r + J] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);  // lo.b2 lo.b3 hi.b2 hi.b3
        } else if constexpr (J == 8) {
            a[r] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);      // lo.b0 hi.b0 lo.b2 hi.b2
            a[r + J] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);  // lo.b1 hi.b1 lo.b3 hi.b3
        } else {
            a[r] = bs_select(lo, hi << J, M << J);
            a[r + J] = bs_select(hi, lo >> J, M);
        }
    }
}

// In place: on entry bit c of a[r] is element (r, c); on exit bit r of a[c]
// is element (r, c).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
    transpose_step<16, 0x0000FFFFu>(a);
    transpose_step<8, 0x00FF00FFu>(a);
    transpose_step<4, 0x0F0F0F0Fu>(a);
    transpose_step<2, 0x33333333u>(a);
    transpose_step<1, 0x55555555u>(a);
}

// (hi:lo) >> (s mod 32); s = 0 gives lo
__device__ __forceinline__ uint32_t bs_funnel(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// Bytes [16k - lead, 16k - lead + 16) of the region [src, src + len)
// (lead = src & 15) one by one, zero outside it: for the units that straddle
// an end of the region, so that no access leaves it.
__device__ __forceinline__ uint4 bs_edge_unit(const uint8_t* __restrict__ src, uint32_t len,
                                           uint32_t lead, uint32_t k) {
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    for (uint32_t b = 0; b < 16u; ++b) {
        const uint32_t rb = 16u * k + b;
        if (rb >= lead && rb < lead + len) v[b >> 2] |= (uint32_t)src[rb - lead] << (8u * (b & 3u));
    }
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// n / d for n, d < 2^16 with m = bs_recip(d): for d >= 2, m = 2^32/d + e
// (0 <= e <= 1) and (n m) >> 32 is exact, since e adds at most n/2^32 < 1/d
// to n/d; d = 1 (m would be 2^32) is marked by m = 0.
__host__ __device__ inline uint32_t bs_recip(uint32_t d) {
    return d <= 1 ? 0u : (uint32_t)(0xffffffffull / d) + 1u;
}
__device__ __forceinline__ uint32_t bs_div(uint32_t n, uint32_t m) { return m ? __umulhi(n, m) : n; }

constexpr uint32_t kElemsPerLane = 3;  // elements per product lane per chunk
constexpr uint32_t kStageRegs = 4;     // 16-byte staging loads per lane per chunk
constexpr uint32_t kChunkBytes = 240;  // most bytes of one pair's chunk (units <= 16)
constexpr uint32_t kChunkElems = 128;  // most elements per chunk (LDS stays below 56 KiB)
constexpr uint32_t kPadBlock = kTile + 1;  // LDS words per 16 planes (one pad word)
constexpr uint32_t kRawSkew = 16;          // extra words before side Y's raw bytes (banks)

// LDS word of plane m of an element laid out in blocks of 16 planes and one
// pad word: tiles of different j-blocks, t-blocks and elements fall in
// different banks.
__host__ __device__ constexpr uint32_t bs_pad(uint32_t m) { return kPadBlock * (m >> 4) + (m & 15u); }

// Whether the diagonal tiles are folded (one lane takes both triangles).  It
// saves a sixth of the products at q = 80 but holds 16 more registers per
// lane; measured on MI355X over q = 32 .. 112, it pays from q = 96 on.
__host__ __device__ constexpr bool bs_fold(uint32_t q) { return q % kTile == 0 && q >= 96; }

// Geometry of the kernel for (q, n_e) and a work-group of nt lanes, computed
// once per launch on the host and passed to the kernel.  Elements are
// processed in chunks of ec: each chunk's bytes are staged raw, transposed
// into planes, multiplied.
struct BsGeom {
    uint32_t qb, qw, jp, xs, ys;
    uint32_t jb_n, tb_n, reach, n_pos;  // product tiles: positions (j-block, offset)
    uint32_t fold;                      // 1: q % 16 == 0, diagonal tiles carry the last offset
    uint32_t subsets, ec, units;        // element subsets, chunk elements, 16-byte units
    uint32_t raw, xp, yp, cp, zp, ot, total;  // LDS word offsets and size
};

inline BsGeom bs_geom(uint32_t q, uint32_t n_e, uint32_t nt) {
    BsGeom g;
    g.qb = q / 8;
    g.qw = (q + 31) / 32;
    g.jp = (q + kTile - 1) / kTile * kTile;
    g.xs = g.jp / kTile * kPadBlock;                    // X: planes 0 .. jp - 1
    // Y: planes -kYLo .. jp + kYHi - 1, element stride odd so that the plane
    // writes of up to 32 elements fall in different banks
    g.ys = (kYLo + g.jp + kYHi) / kTile * kPadBlock + 1;
    g.jb_n = g.jp / kTile;
    g.tb_n = (2 * q - 1 + kTile - 1) / kTile;
    // t-block tb = jb + dt covers t - j from 16 dt - 15 to 16 dt + 15, so dt
    // runs to (q + 14) / 16.  When 16 divides q, the tile at dt = 0 needs only
    // j <= t and the one at dt = q/16 only j > t: one lane takes both halves
    // (256 operations, like a full tile), and dt runs to q/16 - 1.
    g.fold = bs_fold(q) ? 1u : 0u;
    g.reach = g.fold ? q / kTile : (q + 14) / kTile + 1;
    g.n_pos = g.jb_n * g.reach;           // at most 72 (q = 120)
    uint32_t s = nt / g.n_pos;
    if (s == 0) s = 1;
    if (s > n_e) s = n_e;
    uint32_t ec = s * kElemsPerLane;
    if (ec > n_e) ec = n_e;
    if (ec > kChunkBytes / g.qb) ec = kChunkBytes / g.qb;
    if (ec > kChunkElems) ec = kChunkElems;
    // the largest chunk whose layout fits 40 KiB (four work-groups on a CU's
    // 160 KiB) while it still holds an element for every subset, and 64 KiB
    for (;;) {
        g.ec = ec;
        g.units = (ec * g.qb + 14) / 16 + 1;  // covers ec*qb bytes at any offset mod 16
        g.raw = 0;                            // [2 sides][32 pairs][4*units], sides kRawSkew
        g.xp = 2 * kBsPairs * 4 * g.units + kRawSkew + 4;  // words apart, + 4 slack words
        g.yp = g.xp + ec * g.xs;              // X planes [ec][xs]
        g.cp = g.yp + ec * g.ys;              // Y planes [ec][ys], plane k at bs_pad(kYLo + k)
        g.zp = g.cp + 2 * g.jp + kTile;       // C [2 jp + kTile]
        g.ot = g.zp + g.jp;                   // Z [jp]
        g.total = g.ot + kBsPairs * g.qw;     // outputs [32][qw]
        if ((g.total * 4u <= 40960u || ec <= s) && g.total * 4u <= 65536u) break;
        if (ec == 1) break;
        --ec;
    }
    if (s > ec) s = ec;
    g.subsets = s;
    return g;
}

// Work-group of nt = 256 lanes over npw <= 32 pairs from pair0; the pairs'
// blocks form one contiguous region of npw*nbytes bytes per side.
// FOLD: the kernel for shapes with bs_fold(q) (two 16-plane sums per lane).
// Four work-groups per CU (4 waves per SIMD): FOLD = false needs no more than
// 128 VGPRs; FOLD = true spills a few registers outside the inner loops.
template <bool FOLD>
__global__ void __launch_bounds__(kThreads, 4)
bitslice_kernel(const uint8_t* __restrict__ x, const uint8_t* __restrict__ y,
                uint8_t* __restrict__ out, uint64_t n_pairs, ExtShape sh, BsGeom g) {
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t q = sh.q, n_e = sh.n_e, nbytes = sh.nbytes;
    const uint32_t qb = g.qb, qw = g.qw, jp = g.jp, xs = g.xs, ys = g.ys, ec = g.ec;
    const uint32_t units = g.units;
    uint32_t* raw = lds + g.raw;
    uint32_t* xp = lds + g.xp;
    uint32_t* yp = lds + g.yp;
    uint32_t* cp = lds + g.cp;
    uint32_t* zp = lds + g.zp;
    uint32_t* ot = lds + g.ot;

    const uint64_t pair0 = (uint64_t)blockIdx.x * kBsPairs;
    if (pair0 >= n_pairs) return;
    const uint32_t npw = n_pairs - pair0 < kBsPairs ? (uint32_t)(n_pairs - pair0) : kBsPairs;
    const uint8_t* xb = x + pair0 * nbytes;
    const uint8_t* yb = y + pair0 * nbytes;
    const uint32_t len = npw * nbytes;
    const uint32_t lead_x = (uint32_t)((uintptr_t)xb & 15u);
    const uint32_t lead_y = (uint32_t)((uintptr_t)yb & 15u);

    for (uint32_t i = tid; i < 2 * jp + kTile; i += nt) cp[i] = 0u;
    for (uint32_t i = tid; i < ec * (kYLo + kYHi); i += nt) {  // Y's zero margins
        const uint32_t e = i / (kYLo + kYHi), r = i - e * (kYLo + kYHi);
        yp[e * ys + bs_pad(r < kYLo ? r : jp + r)] = 0u;  // r >= kYLo: plane jp + (r - kYLo)
    }

    // ---- staging: unit k = (side, pair p, u) of chunk c is the 16-byte unit
    // (lead + p*nbytes + c*ec*qb) / 16 + u of the side's raw region.  Units
    // inside the region are loaded with 16-byte loads; units that straddle an
    // end are read bytewise when stored; units outside it, and of pairs past
    // npw, are zero.
    const uint32_t n_units = 2 * kBsPairs * units;  // <= kStageRegs * nt
    // slot r of this lane: unit k = tid + r*nt, packed as (lead + p*nbytes) << 4 | u
    // (below 2^32: nbytes < 2^23), or ~0 for no unit (k >= n_units or p >= npw)
    const uint32_t rcp_units = bs_recip(units);  // k < 2^11, units <= 16
    uint32_t slot[kStageRegs];
#pragma unroll
    for (uint32_t r = 0; r < kStageRegs; ++r) {
        const uint32_t k = tid + r * nt;
        const uint32_t side = k >= kBsPairs * units ? 1u : 0u;
        const uint32_t rem = k - side * (kBsPairs * units);
        const uint32_t p = bs_div(rem, rcp_units), u = rem - p * units;
        slot[r] = (k < n_units && p < npw) ? ((side ? lead_y : lead_x) + p * nbytes) << 4 | u : ~0u;
    }
    uint4 st[kStageRegs];
    uint32_t edge = 0;  // bit r: slot r's unit straddles an end of the region
    auto unit_index = [&](uint32_t r, uint32_t c) -> uint32_t {
        return (((slot[r] >> 4) + c * ec * qb) >> 4) + (slot[r] & 15u);
    };
    auto load_chunk = [&](uint32_t c) {
        edge = 0;
#pragma unroll
        for (uint32_t r = 0; r < kStageRegs; ++r) {
            st[r] = make_uint4(0u, 0u, 0u, 0u);
            if (slot[r] != ~0u) {
                const uint32_t side = tid + r * nt >= kBsPairs * units ? 1u : 0u;
                const uint32_t lead = side ? lead_y : lead_x;
                const uint32_t uk = unit_index(r, c), first = 16u * uk;
                if (first >= lead && first + 16u <= lead + len)
                    st[r] = reinterpret_cast<const uint4*>((side ? yb : xb) - lead)[uk];
                else if (first < lead + len && first + 16u > lead)
                    edge |= 1u << r;
            }
        }
    };
    auto store_chunk = [&](uint32_t c) {
#pragma unroll
        for (uint32_t r = 0; r < kStageRegs; ++r) {
            const uint32_t k = tid + r * nt;
            if (k < n_units) {
                uint4 v = st[r];
                if (edge & (1u << r)) {
                    const uint32_t side = k >= kBsPairs * units ? 1u : 0u;
                    v = bs_edge_unit(side ? yb : xb, len, side ? lead_y : lead_x, unit_index(r, c));
                }
                reinterpret_cast<uint4*>(raw + (k >= kBsPairs * units ? kRawSkew : 0u))[k] = v;
            }
        }
    };

    // Lane (position (jb, dt), element subset): x planes j = 16 jb + jj, output
    // planes t = 16 (jb + dt) + i.  Terms with j <= t (jj <= i) take y plane
    // 16 da + (i - jj) and go to acc_lo (t-block jb + da); terms with j > t take
    // y plane 16 db + (i - jj) and go to acc_hi (t-block jb + db).  A plain tile
    // has da = db = dt; a folded diagonal tile has da = 0, db = q/16.
    const uint32_t pos = tid % g.n_pos, sub = tid / g.n_pos;
    const uint32_t jb = pos / g.reach, dt = pos - jb * g.reach;
    const uint32_t da = dt, db = (g.fold && dt == 0) ? q / kTile : dt;
    const bool active = sub < g.subsets && jb + dt < g.tb_n;
    // y planes 16 da + m (m = 0 .. 15) at bs_pad(kYLo + 16 da + m) = 17 (da + 1) + m,
    // and 16 db - 15 + m (m = 0 .. 14) at 17 db + 1 + m; all within
    // [-kYLo, jp + kYHi) since 16 db <= q + 14 and jp >= q
    const uint32_t xoff = jb * kPadBlock;
    const uint32_t yoff_a = (da + 1) * kPadBlock, yoff_b = db * kPadBlock + 1;
    // (not folded: da == db, both halves go to acc_lo and acc_hi stays unused)
    uint32_t acc_lo[kTile], acc_hi[FOLD ? kTile : 1];
#pragma unroll
    for (uint32_t i = 0; i < kTile; ++i) acc_lo[i] = 0u;
#pragma unroll
    for (uint32_t i = 0; i < (FOLD ? kTile : 1); ++i) acc_hi[i] = 0u;

    const uint32_t n_chunks = (n_e + ec - 1) / ec;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (uint32_t c = 0; c < n_chunks; ++c) {
        const uint32_t e_cnt = (c + 1) * ec <= n_e ? ec : n_e - c * ec;
        const uint32_t eoff = c * ec * qb;
        // ---- transposes: item (side, word w, element le) gathers word w of
        // element le of the 32 pairs (two LDS words and a funnel shift each;
        // pairs past npw were staged as zero), transposes, and writes planes
        // 32w .. 32w + 31.  Each side's items fill whole waves (padded to 64
        // slots), so the side, and with it the pairs' byte offsets, are uniform
        // across a wave; within a side the items run word-major
        const uint32_t side_items = e_cnt * qw;
        const uint32_t side_slots = (side_items + 63u) & ~63u;
        const uint32_t rcp_e = bs_recip(e_cnt);  // side_items < 2^16
        for (uint32_t it = tid; it < 2 * side_slots; it += nt) {
            const uint32_t side = __builtin_amdgcn_readfirstlane(it >= side_slots ? 1u : 0u);
            const uint32_t r = it - side * side_slots;
            if (r >= side_items) continue;
            const uint32_t w = bs_div(r, rcp_e);  // word-major within the side
            const uint32_t le = r - w * e_cnt;
            const uint32_t* rs = raw + side * (kBsPairs * 4 * units + kRawSkew);
            const uint32_t lead = side ? lead_y : lead_x;
            const uint32_t lt = le * qb + 4u * w;  // byte of the word in the pair's chunk
            uint32_t a[32];
            // both words are always read (the second may be the next pair's
            // or a slack word) so that the 64 reads issue back to back
#pragma unroll
            for (uint32_t h = 0; h < 32; h += 8) {
#pragma unroll
                for (uint32_t p = h; p < h + 8; ++p) {
                    const uint32_t o = ((lead + p * nbytes + eoff) & 15u) + lt;
                    const uint32_t* r2 = rs + p * 4 * units + (o >> 2);
                    a[p] = bs_funnel(r2[1], r2[0], o * 8u);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if (qb - 4u * w < 4u) {  // the element's last word: bytes past q/8 are the next one's
                const uint32_t keep = (1u << (8u * (qb - 4u * w))) - 1u;
#pragma unroll
                for (uint32_t p = 0; p < 32; ++p) a[p] &= keep;
            }
            transpose32(a);
            // plane j = 32w + i at bs_pad(j) (X) or bs_pad(kYLo + j) (Y); planes
            // q .. jp - 1 are zero (masked bytes); 32w + 16 <= jp always
            uint32_t* dst = side ? yp + le * ys + kPadBlock + 2 * kPadBlock * w
                                 : xp + le * xs + 2 * kPadBlock * w;
#pragma unroll
            for (uint32_t i = 0; i < 16; ++i) dst[bs_pad(i)] = a[i];
            if (32u * w + 32u <= jp) {
#pragma unroll
                for (uint32_t i = 16; i < 32; ++i) dst[bs_pad(i)] = a[i];
            }
        }
        __syncthreads();
        // ---- products: c[t] ^= x[j] & y[t - j] over the 16x16 tile
        if (active) {
            for (uint32_t le = sub; le < e_cnt; le += g.subsets) {
                const uint32_t* xe = xp + le * xs + xoff;
                const uint32_t* ya = yp + le * ys + yoff_a;
                const uint32_t* yb2 = yp + le * ys + yoff_b;
                // the two halves one after the other: 16 y planes live at a time
                uint32_t xv[kTile], yv[kTile];
#pragma unroll
                for (uint32_t i = 0; i < kTile; ++i) xv[i] = xe[i];
#pragma unroll
                for (uint32_t m = 0; m < kTile; ++m) yv[m] = ya[m];
#pragma unroll
                for (uint32_t i = 0; i < kTile; ++i)
#pragma unroll
                    for (uint32_t jj = 0; jj <= i; ++jj)
                        acc_lo[i] = bs_and_xor(xv[jj], yv[i - jj], acc_lo[i]);
#pragma unroll
                for (uint32_t m = 0; m < kTile - 1; ++m) yv[m] = yb2[m];
#pragma unroll
                for (uint32_t i = 0; i < kTile; ++i)
#pragma unroll
                    for (uint32_t jj = i + 1; jj < kTile; ++jj) {
                        if constexpr (FOLD)
                            acc_hi[i] = bs_and_xor(xv[jj], yv[i + kTile - 1 - jj], acc_hi[i]);
                        else
                            acc_lo[i] = bs_and_xor(xv[jj], yv[i + kTile - 1 - jj], acc_lo[i]);
                    }
            }
        }
        if (c + 1 < n_chunks) {  // the next chunk's bytes (raw is free after the transposes)
            load_chunk(c + 1);
            store_chunk(c + 1);
        }
        __syncthreads();
    }
    if (active) {  // t-blocks below tb_n + 1 (folded: jb + q/16 <= 2q/16 - 1)
        uint32_t* ca = cp + (jb + da) * kTile;
        uint32_t* cb = cp + (jb + db) * kTile;
#pragma unroll
        for (uint32_t i = 0; i < kTile; ++i) {
            if constexpr (FOLD) {
                if (da == db) {
                    const uint32_t v = acc_lo[i] ^ acc_hi[i];
                    if (v) atomicXor(ca + i, v);
                } else {
                    if (acc_lo[i]) atomicXor(ca + i, acc_lo[i]);
                    if (acc_hi[i]) atomicXor(cb + i, acc_hi[i]);
                }
            } else {
                if (acc_lo[i]) atomicXor(ca + i, acc_lo[i]);
            }
        }
    }
    __syncthreads();

    // ---- reduction modulo P ------------------------------------------
    // C = C_lo + t^q H with H[i] = c[q + i] (i <= q - 2) and t^q = 1 + sum_f t^f
    // (every tap f <= q/2).  t^f H = (t^f H mod t^q) + t^q U_f with U_f[i] =
    // H[i + q - f] = c[2q + i - f] for i <= f - 2; D = sum_f U_f; t^q D = D +
    // sum_g t^g D needs no further reduction.  Output plane t < q:
    //   z[t] = c[t] + H[t] + sum_f H[t - f] + D[t] + sum_g D[t - g].
    for (uint32_t t = tid; t < q; t += nt) {
        uint32_t z = cp[t] ^ (t + 1 < q ? cp[q + t] : 0u);
        for (uint32_t k = 0; k < sh.n_taps; ++k) {
            const uint32_t f = sh.taps[k];
            if (t >= f) z ^= cp[q + t - f];                  // (t^f H)[t], t - f <= q - 2
            if (t + 1 < f) z ^= cp[2 * q + t - f];           // U_f[t] in D[t]
            for (uint32_t k2 = 0; k2 < sh.n_taps; ++k2) {    // U_f[t - g] in (t^g D)[t]
                const uint32_t gg = sh.taps[k2];
                if (t >= gg && t - gg + 1 < f) z ^= cp[2 * q + (t - gg) - f];
            }
        }
        zp[t] = z;
    }
    __syncthreads();

    // ---- output: lane w transposes planes 32w .. 32w + 31 into word w of
    // the 32 outputs; then the work-group stores its npw*qb bytes
    for (uint32_t w = tid; w < qw; w += nt) {
        uint32_t a[32];
#pragma unroll
        for (uint32_t i = 0; i < 32; ++i) a[i] = 32u * w + i < q ? zp[32u * w + i] : 0u;
        transpose32(a);  // a[p] = word w of pair p's output
#pragma unroll
        for (uint32_t p = 0; p < 32; ++p) ot[p * qw + w] = a[p];
    }
    __syncthreads();
    uint8_t* ob = out + pair0 * qb;
    for (uint32_t i = tid; i < npw * qb; i += nt) {
        const uint32_t p = i / qb, k = i - p * qb;
        ob[i] = (uint8_t)(ot[p * qw + (k >> 2)] >> (8u * (k & 3u)));
    }
}

}  // namespace

void bitslice_describe(const ExtShape& s, uint32_t* chunk_elements, uint32_t* tile_positions,
                       uint32_t* element_subsets, uint32_t* folded) {
    const BsGeom g = bs_geom(s.q, s.n_e, kThreads);
    *chunk_elements = g.ec;
    *tile_positions = g.n_pos;
    *element_subsets = g.subsets;
    *folded = g.fold;
}

uint32_t bitslice_lds_words(const ExtShape& s) {
    if (s.q == 0 || s.q % 8 || s.q > kBitsliceMaxQ || s.n_e == 0) return 0xffffffffu;
    return bs_geom(s.q, s.n_e, kThreads).total;
}

hipError_t launch_bitslice(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                           uint64_t n_pairs, hipStream_t stream) {
    if (n_pairs == 0) return hipSuccess;
    if (s.q == 0 || s.q > kBitsliceMaxQ || s.q % 8 || s.n_e == 0) return hipErrorInvalidValue;
    if ((uint64_t)s.nbytes * 8 != (uint64_t)s.q * s.n_e || s.nbytes >= (1u << 23))
        return hipErrorInvalidValue;
    const BsGeom g = bs_geom(s.q, s.n_e, kThreads);
    if (g.n_pos > (uint32_t)kThreads || 2 * kBsPairs * g.units > kStageRegs * (uint32_t)kThreads)
        return hipErrorInvalidValue;
    const uint64_t groups = (n_pairs + kBsPairs - 1) / kBsPairs;
    if (groups > 0x7fffffffull) return hipErrorInvalidValue;
    const uint32_t lds = g.total * 4u;
    if (lds > 65536u) return hipErrorInvalidValue;
    if (bs_fold(s.q))
        hipLaunchKernelGGL(bitslice_kernel<true>, dim3((uint32_t)groups), dim3(kThreads), lds,
                           stream, x, y, out, n_pairs, s, g);
    else
        hipLaunchKernelGGL(bitslice_kernel<false>, dim3((uint32_t)groups), dim3(kThreads), lds,
                           stream, x, y, out, n_pairs, s, g);
    return hipGetLastError();
}

}  // namespace qext
