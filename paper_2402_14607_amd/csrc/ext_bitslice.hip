// ext_bitslice.hip -- bit-sliced kernel for small fields (q <= 128) with many
// elements per block, such as the paper's own point (71 elements of F_2^80).
//
// A word-level product of q <= 128 bits spends most of its issue slots on
// shifts and masks.  Here a work-group takes 32 block pairs and transposes
// them so that bit p of a 32-bit "plane" word belongs to pair p: plane (e, j)
// holds bit j of element e of all 32 pairs.  A carry-less product of planes
//     c[t] ^= x[j] & y[t - j]      (one v_bitop3_b32 per (j, t), 32 pairs at once)
// needs no shift and no mask.  The element products are summed as the
// inner product of Def. 3.2 asks, reduced modulo P plane by plane, and
// transposed back into q-bit outputs.
//
// Products.  The q-plane operands are split by L Karatsuba levels into
// pieces of h = q / 2^L planes.  Sub-product s = (s_1 .. s_L), each digit lo,
// hi or lo+hi, multiplies the matching piece combinations of x and y
// (h x h planes: h^2 AND-XORs); 3^L of them replace the q^2 schoolbook terms
// (q = 80, L = 2: 9 x 400 = 3600 instead of 6400).  Every lane owns one
// sub-product and an element subset, keeps its 2h - 1 product planes in
// registers across all elements (the inner product's sum commutes with the
// Karatsuba recombination, which therefore runs once per 32 pairs).  An
// operand pass after the transposes writes, per element and side, every
// operand that XORs two or more pieces next to the raw planes, so that the
// product lanes only read their two h-plane operands.
//
// Transposes.  Item (side, half hp, word w) reads 32-bit word w of the
// chunk's byte stream of the 16 pairs 16hp .. 16hp + 15 straight from memory
// (buffer loads, bounds-checked against the work-group's region, so that
// pairs past the last one read zero), transposes the 16 x 32 bit matrix
// (both 16 x 16 halves at once) and writes its 16-bit halves of stream
// planes 32w .. 32w + 31.  The elements are taken in chunks (the paper's
// point: 28 elements, one per element subset, 40.5 KB of operand slots);
// work-groups are persistent over 32-pair groups, and a chunk's rows are
// loaded into registers while the chunk before it multiplies.
//
// After the last chunk the lanes store their sums in LDS, the element
// subsets' sums are added per sub-product, the sub-products recombined level
// by level into the 2q - 1 product planes, reduced modulo P (two folding
// passes, taps at most q/2), and lane (pair p, word w) gathers bit p of
// planes 32w .. 32w + 31 into its output word.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <unordered_map>

#include "ext_internal.h"

namespace qext {
namespace {

constexpr uint32_t kBsPairs = 32;      // pairs per work-group (bits of a plane)
constexpr uint32_t kMaxLevels = 3;
constexpr uint32_t kMaxSub = 27;       // 3^kMaxLevels
constexpr uint32_t kMaxPiece = 20;     // largest piece size h (registers: 4h - 1 per lane)
constexpr uint32_t kLdsTarget = 53248;  // three work-groups on a CU's 160 KiB
constexpr uint32_t kMaxTaps = 3;
constexpr uint32_t kMaxIpl = 2;        // transpose items per lane per chunk (held in registers)
// third word of a buffer resource: 32-bit data format, no swizzle, stride 0
constexpr int kBufferConfig = 0x00020000;

constexpr uint32_t pow3(uint32_t l) { return l == 0 ? 1u : 3u * pow3(l - 1); }

__device__ __forceinline__ uint32_t bs_and_xor(uint32_t a, uint32_t b, uint32_t acc) {
    return __builtin_amdgcn_bitop3_b32(a, b, acc, 0x6A);  // (a & b) ^ acc
}

// One block-swap step of a bit transpose: for rows r with bit J clear, the
// columns of row r with bit J set are exchanged with the columns of row
// r + J with bit J clear (M selects the columns with bit J clear).  The step
// of 8 moves whole bytes (one v_perm_b32 per row); the others take a shift
// and a bit select (v_bitop3_b32 0xD8: (a & ~m) | (b & m)) per row.
__device__ __forceinline__ uint32_t bs_select(uint32_t a, uint32_t b, uint32_t m) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0xD8);
}

template <int J, uint32_t M, int N>
__device__ __forceinline__ void transpose_step(uint32_t (&a)[N]) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
        if (r & J) continue;
        const uint32_t lo = a[r], hi = a[r + J];
        if constexpr (J == 8) {
            a[r] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);      // lo.b0 hi.b0 lo.b2 hi.b2
            a[r + J] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);  // lo.b1 hi.b1 lo.b3 hi.b3
        } else {
            a[r] = bs_select(lo, hi << J, M << J);
            a[r + J] = bs_select(hi, lo >> J, M);
        }
    }
}

// 16 rows, both 16-bit halves at once: on entry bit c of a[r] is element
// (r, c) of a 16 x 32 matrix; on exit bit r of the low half of a[c] is
// element (r, c) and bit r of the high half is element (r, 16 + c).
__device__ __forceinline__ void transpose16(uint32_t (&a)[16]) {
    transpose_step<8, 0x00FF00FFu>(a);
    transpose_step<4, 0x0F0F0F0Fu>(a);
    transpose_step<2, 0x33333333u>(a);
    transpose_step<1, 0x55555555u>(a);
}

// n / d for n, d < 2^16 with m = bs_recip(d): for d >= 2, m = 2^32/d + e
// (0 <= e <= 1) and (n m) >> 32 is exact, since e adds at most n/2^32 < 1/d
// to n/d; d = 1 (m would be 2^32) is marked by m = 0.
__host__ __device__ inline uint32_t bs_recip(uint32_t d) {
    return d <= 1 ? 0u : (uint32_t)(0xffffffffull / d) + 1u;
}
__device__ __forceinline__ uint32_t bs_div(uint32_t n, uint32_t m) {
    return m ? __umulhi(n, m) : n;
}

// Number of lo+hi digits of sub-product s (base-3 digits, 2 = lo+hi).
__host__ __device__ constexpr uint32_t bs_sums(uint32_t s, uint32_t levels) {
    uint32_t n = 0;
    for (uint32_t l = 0; l < levels; ++l, s /= 3) n += s % 3 == 2 ? 1u : 0u;
    return n;
}

// Operand slots of one element (one side) in LDS: the 2^L pieces in their
// natural order (the element's q raw planes), then the 3^L - 2^L operands
// that XOR two or more pieces, in the order of their sub-product index.
// Slot of sub-product s, in units of h planes.
__host__ __device__ constexpr uint32_t bs_slot(uint32_t s, uint32_t levels) {
    uint32_t piece = 0, sum = 0, rest = s;
    for (uint32_t b = 0; b < levels; ++b, rest /= 3) {  // digit of level L - b: piece bit b
        if (rest % 3 == 1) piece |= 1u << b;
        if (rest % 3 == 2) sum = 1;
    }
    if (!sum) return piece;
    uint32_t k = 0;  // sums among the sub-products before s
    for (uint32_t t = 0; t < s; ++t) k += bs_sums(t, levels) ? 1u : 0u;
    return (1u << levels) + k;
}

// Geometry of a launch for (q, n_e), computed once on the host and passed
// to the kernel by value.
struct BsGeom {
    uint32_t qb, qw, es;       // bytes, words per element; LDS words per element's slots
    uint32_t levels, h, n_sub, subsets;
    uint32_t ec;               // elements per chunk (the last chunk may hold fewer)
    uint32_t xp, yp;           // chunk phase: LDS word offsets of the X and Y slots
    uint32_t ss;               // end phase: words per lane-sum row [n_sub][2h - 1] (odd)
    uint32_t pa, pb, zp;       // end phase: recombination buffers, Z
    uint32_t total;            // LDS words
    uint32_t rcp_q;            // bs_recip(q)
};

// The layout of (q, n_e) with L levels and chunks of ec elements.
BsGeom bs_layout(uint32_t q, uint32_t n_e, uint32_t levels, uint32_t ec) {
    BsGeom g{};
    g.qb = q / 8;
    g.qw = (q + 31) / 32;
    g.levels = levels;
    g.h = q >> levels;
    g.n_sub = pow3(levels);
    g.subsets = kThreads / g.n_sub;
    g.es = (g.n_sub * g.h) | 1u;  // odd: consecutive elements fall in different banks
    g.ec = ec < n_e ? ec : n_e;
    g.xp = 0;
    g.yp = g.ec * g.es;
    const uint32_t chunk_total = 2 * g.ec * g.es;
    // end phase: lane sums [subset][ss] from word 0, the subset sums at pa
    // after them; once those are added up, the lane sums are dead and the
    // recombination's second buffer pb and Z (padded to whole words of
    // planes) reuse their words
    g.ss = (g.n_sub * (2 * g.h - 1)) | 1u;
    g.pa = g.subsets * g.ss;
    g.pb = 0;
    g.zp = g.n_sub * 2 * g.h;
    const uint32_t end_total = g.pa + g.n_sub * 2 * g.h;
    g.total = end_total > chunk_total ? end_total : chunk_total;
    g.rcp_q = bs_recip(q);
    return g;
}

// Estimated wave64 instructions issued per 32 pairs of a layout: the
// product rounds (h^2 AND-XORs and, at half weight, the 2h operand reads of
// every active wave), the operand pass (per element and side, the XORs of
// the sum operands and, at half weight, the reads and writes), the
// transposes (one wave per 64 words of each side and half of a chunk's
// stream), and the end phase.
double bs_cost(const BsGeom& g, uint32_t n_e) {
    const uint32_t lanes = g.n_sub * g.subsets;
    const double round = ((lanes + 63) / 64) * (g.h * g.h + g.h + 16.0);
    const uint32_t q = g.qb * 8;
    uint32_t xors = 0;
    for (uint32_t s = 0; s < g.n_sub; ++s) xors += (1u << bs_sums(s, g.levels)) - 1u;
    const double per_elem = 2.0 * g.h * (xors + 0.5 * g.n_sub) / 64.0;  // reads + writes
    auto chunk = [&](uint32_t e) {
        const uint32_t words = (e * q + 31) / 32;
        return ((e + g.subsets - 1) / g.subsets) * round + e * per_elem +
               4.0 * ((words + 63) / 64) * 200.0 + 300.0;
    };
    const double end = 4.0 * (2.0 * g.h + 2.0 * g.subsets) + 2.0 * 200.0;
    return (n_e / g.ec) * chunk(g.ec) + (n_e % g.ec ? chunk(n_e % g.ec) : 0.0) + end;
}

// The layout the kernel runs for (q, n_e): over the Karatsuba depths whose
// pieces fit the registers (8 <= h <= kMaxPiece, or h = q below 8), the
// cheapest by bs_cost, each depth with the fewest equal chunks whose planes
// fit kLdsTarget and whose words fit kMaxIpl items per lane.
BsGeom bs_search(uint32_t q, uint32_t n_e) {
    BsGeom best{};
    double best_cost = 0.0;
    bool have = false;
    for (uint32_t levels = 0; levels <= kMaxLevels; ++levels) {
        if (q % (1u << levels) || (q >> levels) > kMaxPiece) continue;
        if (levels > 0 && (q >> levels) < 8) break;
        for (uint32_t ec = 1; ec <= n_e && ec <= 4096; ++ec) {
            if ((ec * q + 31) / 32 > 64 * kMaxIpl) break;
            const BsGeom g = bs_layout(q, n_e, levels, ec);
            if (g.total * 4 > kLdsTarget) break;
            const double cost = bs_cost(g, n_e);
            if (!have || cost < best_cost) best = g, best_cost = cost, have = true;
        }
    }
    return best;
}

// bs_search, remembered per (q, n_e) for the life of the process.
BsGeom bs_geom(uint32_t q, uint32_t n_e) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, BsGeom> seen;
    const uint64_t key = (uint64_t)q << 32 | n_e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = seen.find(key);
    if (it == seen.end()) it = seen.emplace(key, bs_search(q, n_e)).first;
    return it->second;
}

// One task (a chunk of one 32-pair group) as the transposes see it.  The
// chunk's byte stream of each side and half (pairs 16*half .. 16*half + 15)
// is cut into waves of 64 words: lane l of item-wave (side, half, j)
// transposes word w = 64j + 2(l mod 32) + l / 32 (each half-wave takes every
// other word, which spreads its 16-bit plane stores over about twice as many
// LDS banks as consecutive words would).  Item-wave iw = wave + 4m (m < nw) of the
// work-group's four waves has (side, half) = iw / nw and j = iw mod nw, so
// every lane holds nw items, nw <= kMaxIpl.
struct BsTask {
    const uint8_t* base_x;  // dword holding the first byte of each side's region
    const uint8_t* base_y;
    uint32_t nrec_x, nrec_y;  // buffer lengths: lead + region bytes, whole dwords
    uint32_t lead_x, lead_y;  // first byte's offset in its dword
    uint32_t eoff;            // the chunk's first byte in a block
    uint32_t bits, words, nw; // the chunk's stream bits and words; item-waves per (side, half)
};

__device__ __forceinline__ BsTask bs_task(const uint8_t* x, const uint8_t* y, uint64_t n_pairs,
                                          uint32_t nbytes, uint32_t q, uint32_t ec, uint32_t n_e,
                                          uint32_t group, uint32_t chunk) {
    BsTask t;
    const uint64_t pair0 = (uint64_t)group * kBsPairs;
    const uint32_t npw = n_pairs - pair0 < kBsPairs ? (uint32_t)(n_pairs - pair0) : kBsPairs;
    const uint32_t len = npw * nbytes;
    const uintptr_t ax = (uintptr_t)(x + pair0 * nbytes), ay = (uintptr_t)(y + pair0 * nbytes);
    t.lead_x = (uint32_t)(ax & 3u);
    t.lead_y = (uint32_t)(ay & 3u);
    t.base_x = (const uint8_t*)(ax - t.lead_x);
    t.base_y = (const uint8_t*)(ay - t.lead_y);
    t.nrec_x = (t.lead_x + len + 3) & ~3u;
    t.nrec_y = (t.lead_y + len + 3) & ~3u;
    const uint32_t e_cnt = (chunk + 1) * ec <= n_e ? ec : n_e - chunk * ec;
    t.eoff = chunk * ec * (q / 8);
    t.bits = e_cnt * q;
    t.words = (t.bits + 31) / 32;
    t.nw = (t.words + 63) / 64;
    return t;
}

// Byte offset of row p's chunk stream (p = 0..15 of half hf) in its side's buffer.
__device__ __forceinline__ uint32_t bs_row(const BsTask& t, uint32_t nbytes, bool side_y,
                                           uint32_t hf, uint32_t p) {
    return (side_y ? t.lead_y : t.lead_x) + (hf * 16u + p) * nbytes + t.eoff;
}

// Loads the task's items: for each row, the two dwords that word w
// straddles, one 8-byte load from a buffer that starts at the row's first
// dword (the lanes' offsets are just 4w).  The buffer is bounds-checked per
// dword against the region's end, so rows of pairs past the last read zero
// and a pair of dwords whose second one lies past the end still returns the
// first.
template <uint32_t IPL>
__device__ __forceinline__ void bs_load_task(const BsTask& t, uint32_t nbytes, uint32_t wave,
                                             uint32_t lane, uint32_t (&lo)[IPL][16],
                                             uint32_t (&hi)[IPL][16]) {
#pragma unroll
    for (uint32_t m = 0; m < IPL; ++m) {
        if (m >= t.nw) break;
        const uint32_t iw = wave + 4u * m;
        const uint32_t sh2 = iw / t.nw, j = iw - sh2 * t.nw;
        const bool side_y = (sh2 >> 1) != 0;
        const uint8_t* base = side_y ? t.base_y : t.base_x;
        const uint32_t nrec = side_y ? t.nrec_y : t.nrec_x;
        const uint32_t w = 64u * j + 2u * (lane & 31u) + (lane >> 5);
#pragma unroll
        for (uint32_t p = 0; p < 16; ++p) {
            // row start and length as scalars (the resource must be uniform)
            const uint32_t row = bs_row(t, nbytes, side_y, sh2 & 1u, p);
            const uint32_t rs = __builtin_amdgcn_readfirstlane(row & ~3u);
            const uint32_t n = __builtin_amdgcn_readfirstlane(nrec > rs ? nrec - rs : 0u);
            const __amdgpu_buffer_rsrc_t res = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(base + rs), (short)0, (int)n, kBufferConfig);
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(res, 4u * w, 0, 0);
            lo[m][p] = v[0];
            hi[m][p] = v[1];
        }
    }
}

// Transposes the task's items and writes their 16-bit halves of stream
// planes 32w .. 32w + 31 (plane b is bit b mod q of element b / q) in
// groups of 8 (q is a multiple of 8).
template <uint32_t IPL>
__device__ __forceinline__ void bs_put_task(const BsTask& t, uint32_t nbytes, uint32_t wave,
                                            uint32_t lane, const uint32_t (&lo)[IPL][16],
                                            const uint32_t (&hi)[IPL][16],
                                            uint32_t* xp, uint32_t* yp, uint32_t es, uint32_t q,
                                            uint32_t rcp_q) {
#pragma unroll
    for (uint32_t m = 0; m < IPL; ++m) {
        if (m >= t.nw) break;
        const uint32_t iw = wave + 4u * m;
        const uint32_t sh2 = iw / t.nw, j = iw - sh2 * t.nw;
        const bool side_y = (sh2 >> 1) != 0;
        const uint32_t w = 64u * j + 2u * (lane & 31u) + (lane >> 5);
        uint32_t a[16];
#pragma unroll
        for (uint32_t p = 0; p < 16; ++p) {
            const uint32_t row = bs_row(t, nbytes, side_y, sh2 & 1u, p);
            a[p] = __builtin_amdgcn_alignbit(hi[m][p], lo[m][p], (row & 3u) * 8u);
        }
        if (w >= t.words) continue;
        transpose16(a);  // a[i]: plane i (low half), plane 16 + i (high half)
        uint16_t* planes = reinterpret_cast<uint16_t*>(side_y ? yp : xp) + (sh2 & 1u);
#pragma unroll
        for (uint32_t gi = 0; gi < 4; ++gi) {
            const uint32_t b = 32u * w + 8u * gi;
            if (b < t.bits) {
                const uint32_t e = bs_div(b, rcp_q);
                uint16_t* dst = planes + 2 * (e * es + (b - e * q));
#pragma unroll
                for (uint32_t i = 0; i < 8; ++i) {
                    const uint32_t v = a[8 * (gi & 1u) + i];
                    dst[2 * i] = (uint16_t)(gi < 2 ? v : v >> 16);
                }
            }
        }
    }
}

// The operand pass for one position (element, plane i) of one side: reads
// the 2^L pieces' plane i and writes plane i of every operand that XORs two
// or more of them (base points at plane i of the element's slots).  Piece p
// belongs to sub-product s when each of s's lo/hi digits matches p's bit.
template <uint32_t H, uint32_t L>
__device__ __forceinline__ void bs_form(uint32_t* base) {
    constexpr uint32_t kPieces = 1u << L;
    uint32_t pc[kPieces];
#pragma unroll
    for (uint32_t p = 0; p < kPieces; ++p) pc[p] = base[p * H];
#pragma unroll
    for (uint32_t s = 0; s < pow3(L); ++s) {
        if (bs_sums(s, L) == 0) continue;
        uint32_t v = 0;
#pragma unroll
        for (uint32_t p = 0; p < kPieces; ++p) {
            bool match = true;
            uint32_t rest = s;
#pragma unroll
            for (uint32_t b = 0; b < L; ++b, rest /= 3) {
                if (rest % 3 == 0 && (p >> b & 1u)) match = false;
                if (rest % 3 == 1 && !(p >> b & 1u)) match = false;
            }
            if (match) v ^= pc[p];
        }
        base[bs_slot(s, L) * H] = v;
    }
}

// cp[idx] if on, else 0, reading cp[0] instead: the read is always in range.
__device__ __forceinline__ uint32_t bs_term(const uint32_t* cp, bool on, uint32_t idx) {
    return cp[on ? idx : 0u] & (on ? ~0u : 0u);
}

// Work-group of 256 lanes, persistent over 32-pair groups; each group's
// blocks form one contiguous region of npw*nbytes bytes per side, at any
// byte offset.  H: piece size h, L: Karatsuba levels (q = H * 2^L).  Three
// work-groups per CU (at most 168 VGPRs per lane).
template <uint32_t H, uint32_t L>
__global__ void __launch_bounds__(kThreads, 3)
bitslice_kernel(const uint8_t* __restrict__ x, const uint8_t* __restrict__ y,
                uint8_t* __restrict__ out, uint64_t n_pairs, ExtShape sh, BsGeom g) {
    constexpr uint32_t kAcc = 2 * H - 1;
    constexpr uint32_t kSub = pow3(L);
    constexpr uint32_t kSubsets = kThreads / kSub;
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / 64u), lane = tid & 63u;
    const uint32_t q = sh.q, n_e = sh.n_e, nbytes = sh.nbytes;
    const uint32_t qb = g.qb, es = g.es, ec = g.ec;
    uint32_t* xp = lds + g.xp;
    uint32_t* yp = lds + g.yp;
    const uint32_t n_groups = (uint32_t)((n_pairs + kBsPairs - 1) / kBsPairs);
    const uint32_t n_chunks = (n_e + ec - 1) / ec;

    // Lane (sub-product s, element subset): its operands are slot bs_slot(s)
    // of each element of X and Y
    const uint32_t s = tid / kSubsets, sub = tid - s * kSubsets;
    const bool active = s < kSub;
    const uint32_t off0 = active ? bs_slot(s, L) * H : 0u;
    uint32_t acc[kAcc];
#pragma unroll
    for (uint32_t i = 0; i < kAcc; ++i) acc[i] = 0u;

    // Persistent: the work-group takes groups blockIdx.x, + gridDim.x, ...,
    // each chunk by chunk.  A task's items are loaded into registers while
    // the task before it multiplies (and, after a group's last chunk, sums,
    // reduces and stores), so that its transposes find them there.
    uint32_t group = blockIdx.x, chunk = 0;
    if (group >= n_groups) return;
    uint32_t rows_lo[kMaxIpl][16], rows_hi[kMaxIpl][16];
    BsTask cur = bs_task(x, y, n_pairs, nbytes, q, ec, n_e, group, chunk);
    bs_load_task<kMaxIpl>(cur, nbytes, wave, lane, rows_lo, rows_hi);
#pragma unroll 1
    for (;;) {
        bs_put_task<kMaxIpl>(cur, nbytes, wave, lane, rows_lo, rows_hi, xp, yp, es, q, g.rcp_q);
        __syncthreads();
        const uint32_t e_cnt = cur.bits / q;
        if constexpr (L > 0) {
            // ---- operand pass: the sum operands of every element and side
            for (uint32_t pos = tid; pos < e_cnt * H; pos += nt) {
                const uint32_t e = pos / H, i = pos - e * H;
                bs_form<H, L>(xp + e * es + i);
                bs_form<H, L>(yp + e * es + i);
            }
            __syncthreads();
        }
        const bool last_chunk = chunk + 1 == n_chunks;
        const uint32_t next_group = last_chunk ? group + gridDim.x : group;
        const uint32_t next_chunk = last_chunk ? 0u : chunk + 1;
        const bool more = next_group < n_groups;
        BsTask nxt = cur;
        if (more) {
            nxt = bs_task(x, y, n_pairs, nbytes, q, ec, n_e, next_group, next_chunk);
            bs_load_task<kMaxIpl>(nxt, nbytes, wave, lane, rows_lo, rows_hi);
        }
        // ---- products: the lane's sub-product over its elements of the chunk
#pragma unroll 1
        for (uint32_t le = active ? sub : e_cnt; le < e_cnt; le += kSubsets) {
            const uint32_t* xe = xp + le * es + off0;
            const uint32_t* ye = yp + le * es + off0;
            uint32_t xv[H], yv[H];
#pragma unroll
            for (uint32_t i = 0; i < H; ++i) xv[i] = xe[i];
#pragma unroll
            for (uint32_t i = 0; i < H; ++i) yv[i] = ye[i];
#pragma unroll
            for (uint32_t kk = 0; kk < H; ++kk)
#pragma unroll
                for (uint32_t j = 0; j < H; ++j)
                    acc[j + kk] = bs_and_xor(xv[j], yv[kk], acc[j + kk]);
        }
        __syncthreads();  // the planes are read before the next chunk or the sums overwrite them
        if (last_chunk) {
            const uint64_t pair0 = (uint64_t)group * kBsPairs;
            const uint32_t npw =
                n_pairs - pair0 < kBsPairs ? (uint32_t)(n_pairs - pair0) : kBsPairs;
            // ---- sums: lane (rank, subset) stores its sums at row `subset`, column
            // s*(2H - 1) of [subsets][ss] (ss odd: the subsets of a sub-product fall
            // in different banks); then each (s, t) is the XOR over the subsets
            if (active) {
                uint32_t* dst = lds + sub * g.ss + s * kAcc;
#pragma unroll
                for (uint32_t t = 0; t < kAcc; ++t) dst[t] = acc[t];
            }
            __syncthreads();
            uint32_t* src = lds + g.pa;
            for (uint32_t i = tid; i < kSub * kAcc; i += nt) {
                uint32_t v = 0;
#pragma unroll
                for (uint32_t k = 0; k < kSubsets; ++k) v ^= lds[k * g.ss + i];
                src[i] = v;
            }
            __syncthreads();

            // ---- recombination, innermost level first: the product of operands
            // split as a + z^n b (pieces of n planes) is
            //   ab = A (1 + z^n) + M z^n + B (z^n + z^2n)
            // with A = a_lo b_lo, B = a_hi b_hi, M = (a_lo + a_hi)(b_lo + b_hi); the
            // children of product s' are 3s' + {0: lo, 1: hi, 2: lo+hi}
            {
                uint32_t* dst = lds + g.pb;
                uint32_t n = kSub, size = H;
#pragma unroll
                for (uint32_t l = 0; l < L; ++l) {
                    const uint32_t in_w = 2 * size - 1, out_w = 4 * size - 1;
                    n /= 3;
                    for (uint32_t i = tid; i < n * out_w; i += nt) {
                        const uint32_t sp = i / out_w, t = i - sp * out_w;
                        const uint32_t* lo = src + 3 * sp * in_w;
                        const uint32_t* hi = lo + in_w;
                        const uint32_t* mid = hi + in_w;
                        // every read in range (indices clamped), terms outside their
                        // window masked off, so that the reads issue together
                        const uint32_t t1 = t >= size ? t - size : 0u;
                        const uint32_t t2 = t >= 2 * size ? t - 2 * size : 0u;
                        const uint32_t m0 = t < in_w ? ~0u : 0u;
                        const uint32_t m1 = t >= size && t1 < in_w ? ~0u : 0u;
                        const uint32_t m2 = t >= 2 * size && t2 < in_w ? ~0u : 0u;
                        const uint32_t c0 = t < in_w ? t : 0u, c1 = t1 < in_w ? t1 : 0u;
                        const uint32_t c2 = t2 < in_w ? t2 : 0u;
                        dst[i] = (lo[c0] & m0) ^ ((lo[c1] ^ hi[c1] ^ mid[c1]) & m1) ^ (hi[c2] & m2);
                    }
                    __syncthreads();
                    uint32_t* tmp = src;
                    src = dst;
                    dst = tmp;
                    size *= 2;
                }
            }
            const uint32_t* cp = src;  // the 2q - 1 product planes
            uint32_t* zp = lds + g.zp;

            // ---- reduction modulo P ------------------------------------------
            // C = C_lo + t^q H with H[i] = c[q + i] (i <= q - 2) and t^q = 1 + sum_f t^f
            // (every tap f <= q/2).  t^f H = (t^f H mod t^q) + t^q U_f with U_f[i] =
            // H[i + q - f] = c[2q + i - f] for i <= f - 2; D = sum_f U_f; t^q D = D +
            // sum_g t^g D needs no further reduction.  Output plane t < q:
            //   z[t] = c[t] + H[t] + sum_f H[t - f] + D[t] + sum_g D[t - g].
            // Every read is in range (indices clamped into [0, 2q - 1)) and the
            // terms outside their condition are masked off, so that a lane's reads
            // issue together.  Planes q .. 32*qw - 1 of Z are zero.
            for (uint32_t t = tid; t < 32 * g.qw; t += nt) {
                if (t >= q) {
                    zp[t] = 0u;
                    continue;
                }
                uint32_t z = cp[t] ^ bs_term(cp, t + 1 < q, q + t);
#pragma unroll
                for (uint32_t k = 0; k < kMaxTaps; ++k) {
                    const bool tk = k < sh.n_taps;
                    const uint32_t f = tk ? sh.taps[k] : 0u;
                    z ^= bs_term(cp, tk && t >= f, q + t - f);         // (t^f H)[t], t - f <= q - 2
                    z ^= bs_term(cp, tk && t + 1 < f, 2 * q + t - f);   // U_f[t] in D[t]
#pragma unroll
                    for (uint32_t k2 = 0; k2 < kMaxTaps; ++k2) { // U_f[t - g] in (t^g D)[t]
                        const bool tg = tk && k2 < sh.n_taps;
                        const uint32_t gg = tg ? sh.taps[k2] : 0u;
                        z ^= bs_term(cp, tg && t >= gg && t - gg + 1 < f, 2 * q + (t - gg) - f);
                    }
                }
                zp[t] = z;
            }
            __syncthreads();

            // ---- output: lane (pair p, word w) gathers bit p of planes 32w ..
            // 32w + 31 (the same planes for every pair: broadcast reads, all issued
            // before the bits are assembled) and stores the word's bytes of pair p's
            // q/8 output bytes
            const uint32_t qw = g.qw;
            for (uint32_t i = tid; i < kBsPairs * qw; i += nt) {
                const uint32_t w = i / kBsPairs, p = i - w * kBsPairs;
                uint32_t v = 0;
#pragma unroll
                for (uint32_t b = 0; b < 32; ++b) v |= ((zp[32u * w + b] >> p) & 1u) << b;
                if (p >= npw) continue;
                uint8_t* ob = out + (pair0 + p) * qb + 4u * w;
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k)
                    if (4u * w + k < qb) ob[k] = (uint8_t)(v >> (8u * k));
            }
#pragma unroll
            for (uint32_t i = 0; i < kAcc; ++i) acc[i] = 0u;
            __syncthreads();  // Z and the sums are read before the next planes overwrite them
        }
        if (!more) break;
        group = next_group;
        chunk = next_chunk;
        cur = nxt;
    }
}

// Launches one work-group per resident slot (CUs x work-groups per CU at
// this LDS size, looked up once per device and size), or one per group when
// there are fewer groups.
template <uint32_t H, uint32_t L>
hipError_t launch_one(const BsGeom& g, uint32_t groups, const uint8_t* x, const uint8_t* y,
                      uint8_t* out, uint64_t n_pairs, const ExtShape& s, hipStream_t stream) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, uint32_t> resident;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint32_t lds = g.total * 4u;
    const uint64_t key = (uint64_t)(uint32_t)dev << 32 | lds;
    uint32_t slots = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = resident.find(key);
        if (it != resident.end()) slots = it->second;
    }
    if (slots == 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bitslice_kernel<H, L>, kThreads,
                                                         lds);
        if (e != hipSuccess) return e;
        slots = (uint32_t)(cus > 0 ? cus : 1) * (uint32_t)(per_cu > 0 ? per_cu : 1);
        std::lock_guard<std::mutex> lock(mu);
        resident[key] = slots;
    }
    const uint32_t grid = groups < slots ? groups : slots;
    hipLaunchKernelGGL((bitslice_kernel<H, L>), dim3(grid), dim3(kThreads), lds, stream, x, y, out,
                       n_pairs, s, g);
    return hipGetLastError();
}

// The instantiation for (h, levels), or an error if there is none: every q
// that is a multiple of 8 up to 128 at each depth bs_search may pick
// (8 <= h <= 20, except h = q itself below 8).
hipError_t launch_for(const BsGeom& g, uint32_t groups, const uint8_t* x, const uint8_t* y,
                      uint8_t* out, uint64_t n_pairs, const ExtShape& s, hipStream_t stream) {
#define BS_CASE(HH, LL)                                                         \
    if (g.h == HH && g.levels == LL)                                            \
        return launch_one<HH, LL>(g, groups, x, y, out, n_pairs, s, stream);
    BS_CASE(8, 0) BS_CASE(16, 0)
    BS_CASE(8, 1) BS_CASE(12, 1) BS_CASE(16, 1) BS_CASE(20, 1)
    BS_CASE(8, 2) BS_CASE(10, 2) BS_CASE(12, 2) BS_CASE(14, 2) BS_CASE(16, 2) BS_CASE(18, 2)
    BS_CASE(20, 2)
    BS_CASE(8, 3) BS_CASE(9, 3) BS_CASE(10, 3) BS_CASE(11, 3) BS_CASE(12, 3) BS_CASE(13, 3)
    BS_CASE(14, 3) BS_CASE(15, 3) BS_CASE(16, 3)
#undef BS_CASE
    return hipErrorInvalidValue;
}

}  // namespace

void bitslice_describe(const ExtShape& s, uint32_t* chunk_elements, uint32_t* levels,
                       uint32_t* piece_planes, uint32_t* element_subsets) {
    const BsGeom g = bs_geom(s.q, s.n_e);
    *chunk_elements = g.ec;
    *levels = g.levels;
    *piece_planes = g.h;
    *element_subsets = g.subsets;
}

uint32_t bitslice_lds_words(const ExtShape& s) {
    if (s.q == 0 || s.q % 8 || s.q > kBitsliceMaxQ || s.n_e == 0) return 0xffffffffu;
    return bs_geom(s.q, s.n_e).total;
}

hipError_t launch_bitslice(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                           uint64_t n_pairs, hipStream_t stream) {
    if (n_pairs == 0) return hipSuccess;
    if (s.q == 0 || s.q > kBitsliceMaxQ || s.q % 8 || s.n_e == 0) return hipErrorInvalidValue;
    if ((uint64_t)s.nbytes * 8 != (uint64_t)s.q * s.n_e || s.nbytes >= (1u << 23))
        return hipErrorInvalidValue;
    uint32_t max_tap = 0;
    for (uint32_t k = 0; k < s.n_taps; ++k) max_tap = s.taps[k] > max_tap ? s.taps[k] : max_tap;
    if (s.n_taps == 0 || s.n_taps > kMaxTaps || 2 * max_tap > s.q) return hipErrorInvalidValue;
    const BsGeom g = bs_geom(s.q, s.n_e);
    if (g.ec == 0 || g.n_sub * g.subsets > (uint32_t)kThreads || g.h << g.levels != s.q)
        return hipErrorInvalidValue;
    const uint64_t groups = (n_pairs + kBsPairs - 1) / kBsPairs;
    if (groups > 0x7fffffffull) return hipErrorInvalidValue;
    if (g.total * 4u > 65536u) return hipErrorInvalidValue;
    return launch_for(g, (uint32_t)groups, x, y, out, n_pairs, s, stream);
}

}  // namespace qext
