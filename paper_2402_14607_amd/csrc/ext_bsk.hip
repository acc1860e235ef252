// ext_bsk.hip -- bit-sliced Karatsuba kernel for fields of 512, 1024 or 2048
// bits (Def. 3.2's inner product over F_2^q, Algorithm 1's blocks).
//
// The word-level kernel multiplies one pair's elements per lane and spends
// about a fifth of its issue slots on the shifts and masks of a word-level
// carry-less product.  Here a work-group takes 32 block pairs and turns them
// sideways (bit p of every plane word is pair p), so that every product term
// is one v_bitop3_b32 for 32 pairs, as in ext_bitslice.hip, and splits each
// element product L Karatsuba levels down to 3^L products of 256 planes.
//
// Per element e of the 32 pairs' blocks (every step ends with a barrier):
//   1. staging: the element's bytes of both sides (32 pairs x q/8 bytes), with
//      16-byte loads issued one element ahead, stored as words (w, pair) at
//      raw[side][33 w + pair];
//   2. transposes: item (side, w) reads word w of the 32 pairs, transposes the
//      32x32 bit matrix in registers and writes planes 32w .. 32w+31 of the
//      side's plane array (bsk_pad layout);
//   3. operands: the sub-products whose operand is a sum of segments get it
//      materialized (one XOR of 2, 4 or 8 planes per plane); the others read
//      their segment of the plane array in place;
//   4. products: lane task (sub-product p, t-block pair k) runs 17 16x16 tiles,
//      tile (tb, jb): acc[i] ^= x[16 jb + jj] & y[16 (tb - jb) + i - jj], with
//      y blocks outside the operand read from a zero block so that every lane
//      runs the same instruction stream; the two t-blocks' sums stay in
//      registers across all elements (the paper's inner product sums the
//      element products before any reduction).
// Then each lane XORs its sums into C at the sub-product's Karatsuba offsets,
// C is reduced modulo P plane by plane (every tap at most q/2), and lane w
// transposes planes 32w .. 32w+31 back into word w of the 32 outputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ext_bits.h"
#include "ext_bsk.h"
#include "ext_internal.h"

namespace qext {
namespace {

// 16 consecutive planes starting at LDS word w (contiguous: a 16-plane block
// never crosses a pad word), as 8 two-word reads.
__device__ __forceinline__ void bsk_load16(uint32_t (&v)[16], const uint32_t* lds, uint32_t w) {
    const uint32_t* s = lds + w;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = s[i];
}

__global__ void __launch_bounds__(448, 2)
bsk_kernel(const uint8_t* __restrict__ x, const uint8_t* __restrict__ y,
           uint8_t* __restrict__ out, uint64_t n_pairs, ExtShape sh, BskGeom g) {
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t q = g.q, qw = g.qw, n_e = sh.n_e, nbytes = sh.nbytes, qb = q / 8;

    const uint64_t pair0 = (uint64_t)blockIdx.x * kBskPairs;
    if (pair0 >= n_pairs) return;
    const uint32_t npw = n_pairs - pair0 < kBskPairs ? (uint32_t)(n_pairs - pair0) : kBskPairs;
    const uint8_t* xb = x + pair0 * nbytes;
    const uint8_t* yb = y + pair0 * nbytes;

    // ---- staging slots: unit k = tid + r nt is (side, pair, u): the 16-byte
    // unit u of the element's q/8 bytes of that pair; pairs past npw are zero
    const uint32_t per_side = kBskPairs * g.units;
    uint4 st[kBskStage];
    auto load_elem = [&](uint32_t e) {
#pragma unroll
        for (uint32_t r = 0; r < kBskStage; ++r) {
            const uint32_t k = tid + r * nt;
            st[r] = make_uint4(0u, 0u, 0u, 0u);
            if (k < 2 * per_side) {
                const uint32_t side = k >= per_side ? 1u : 0u;
                const uint32_t rem = k - side * per_side;
                const uint32_t pp = rem / g.units, u = rem - pp * g.units;
                if (pp < npw) {
                    const uint8_t* src = (side ? yb : xb) + (uint64_t)pp * nbytes +
                                         (uint64_t)e * qb + 16u * u;
                    st[r] = *reinterpret_cast<const uint4*>(src);
                }
            }
        }
    };
    auto store_elem = [&]() {
#pragma unroll
        for (uint32_t r = 0; r < kBskStage; ++r) {
            const uint32_t k = tid + r * nt;
            if (k < 2 * per_side) {
                const uint32_t side = k >= per_side ? 1u : 0u;
                const uint32_t rem = k - side * per_side;
                const uint32_t pp = rem / g.units, u = rem - pp * g.units;
                uint32_t* d = lds + g.raw + side * g.pa + 33u * (4u * u) + pp;
                d[0] = st[r].x;
                d[33] = st[r].y;
                d[66] = st[r].z;
                d[99] = st[r].w;
            }
        }
    };

    // ---- lane task: sub-product p, t-block pair kk (lanes of one kk adjacent)
    const bool active = tid < g.tasks;
    const uint32_t kk = active ? tid / g.np : 0u;
    const uint32_t p = active ? tid - kk * g.np : 0u;
    const BskTask tk = bsk_task(kk);
    const uint32_t xop = g.xbase[p], yop = g.ybase[p];
    uint32_t acc[16], acc2[16];  // the current t-block, the other one
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        acc[i] = 0u;
        acc2[i] = 0u;
    }

    if (tid < 16) lds[g.zero + tid] = 0u;
    load_elem(0);
    for (uint32_t e = 0; e < n_e; ++e) {
        store_elem();
        __syncthreads();
        // ---- transposes: item (side, w) -> planes 32w .. 32w + 31
        for (uint32_t it = tid; it < 2 * qw; it += nt) {
            const uint32_t side = it >= qw ? 1u : 0u;
            const uint32_t w = it - side * qw;
            const uint32_t* rs = lds + g.raw + side * g.pa + 33u * w;
            uint32_t a[32];
#pragma unroll
            for (int pp = 0; pp < 32; ++pp) a[pp] = rs[pp];
            transpose32(a);
            uint32_t* dst = lds + (side ? g.ypl : g.xpl) + bsk_pad(32u * w);
#pragma unroll
            for (int i = 0; i < 32; ++i) dst[i] = a[i];
        }
        __syncthreads();
        if (e + 1 < n_e) load_elem(e + 1);  // in flight during the operands and products
        // ---- operands: item (side, leaf li, plane k), k fastest
        for (uint32_t it = tid; it < 2 * g.n_leaf * kBskBase; it += nt) {
            // (side, li) is the same for the 64 lanes of a wave: 256 items per leaf
            const uint32_t sl = __builtin_amdgcn_readfirstlane(it / kBskBase);
            const uint32_t side = sl >= g.n_leaf ? 1u : 0u;
            const uint32_t li = sl - side * g.n_leaf, kp = it % kBskBase;
            uint32_t hi, mid;
            bsk_path(g.leaf_p[li], g.levels, &hi, &mid);
            const uint32_t* pl = lds + (side ? g.ypl : g.xpl) + bsk_pad(kp);
            uint32_t v = 0u, sub = mid;
            for (;;) {
                v ^= pl[kBskLeaf * (hi | sub)];
                if (sub == 0) break;
                sub = (sub - 1u) & mid;
            }
            lds[(side ? g.ylf : g.xlf) + kBskLeaf * li + bsk_pad(kp)] = v;
        }
        __syncthreads();
        // ---- products: 17 tiles; acc holds t-block tbA's sum until tile nA,
        // then the sums swap places and acc takes t-block tbB (lanes of one
        // task pair kk switch at the same tile, so a wave takes the swap for
        // at most three values of nA)
        if (active) {
            // block addresses, advanced tile by tile: x block jb, y blocks d
            // and d - 1 (d = tb - jb falls by one per tile within a t-block)
            uint32_t jb = tk.jbA0, d = tk.tbA - tk.jbA0;
            auto blk = [](uint32_t base, uint32_t m) { return base + 16u * m + (m >> 1); };
#pragma unroll 1
            for (uint32_t r = 0; r < kBskIters; ++r) {
                if (r == tk.nA) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const uint32_t t = acc[i];
                        acc[i] = acc2[i];
                        acc2[i] = t;
                    }
                    jb = tk.jbB0;
                    d = tk.tbB - tk.jbB0;
                }
                uint32_t xv[16], ya[16], yv[16];
                bsk_load16(xv, lds, blk(xop, jb));
                bsk_load16(ya, lds, d < 16u ? blk(yop, d) : g.zero);
                bsk_load16(yv, lds, d > 0u ? blk(yop, d - 1u) : g.zero);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
#pragma unroll
                    for (int jj = 0; jj <= i; ++jj) acc[i] = bs_and_xor(xv[jj], ya[i - jj], acc[i]);
#pragma unroll
                    for (int jj = i + 1; jj < 16; ++jj)
                        acc[i] = bs_and_xor(xv[jj], yv[16 + i - jj], acc[i]);
                }
                ++jb;
                --d;
            }
            // every lane swapped once: swap back, so that acc holds tbA's sum
            // and acc2 tbB's for the next element
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t t = acc[i];
                acc[i] = acc2[i];
                acc2[i] = t;
            }
        }
        __syncthreads();  // the next element's staging overwrites the leaves
    }

    // ---- C = sum of the sub-products at their Karatsuba offsets; plane c at
    // cpad(c) = c + c/256, so that the 27 lanes of a task, which add at
    // 256-plane offsets that differ by sub-product, hit different banks
    auto cpad = [](uint32_t c) { return c + (c >> 8); };
    for (uint32_t i = tid; i < cpad(2 * q); i += nt) lds[g.cs + i] = 0u;
    __syncthreads();
    if (active) {
        uint32_t hi, mid;
        bsk_path(p, g.levels, &hi, &mid);
        const uint32_t lmask = (1u << g.levels) - 1u;
        const uint32_t hm = hi | mid, lh = lmask & ~mid;
        uint32_t sub = lh;
        for (;;) {
            // planes t < 512 of the sub-product: cpad(256 a + t) = 257 a + cpad(t)
            uint32_t* c = lds + g.cs + (kBskBase + 1u) * (hm + sub);
            uint32_t* ca = c + cpad(16u * tk.tbA);
            uint32_t* cb = c + cpad(16u * tk.tbB);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (acc[i]) atomicXor(ca + i, acc[i]);
                if (acc2[i]) atomicXor(cb + i, acc2[i]);
            }
            if (sub == 0) break;
            sub = (sub - 1u) & lh;
        }
    }
    __syncthreads();

    // ---- reduction modulo P, plane by plane (every tap at most q/2):
    // z[t] = c[t] + H[t] + sum_f H[t - f] + D[t] + sum_g D[t - g], H[i] =
    // c[q + i], D[i] = sum_f c[2q + i - f] over the f with i <= f - 2
    const uint32_t* cp = lds + g.cs;
    for (uint32_t t = tid; t < q; t += nt) {
        uint32_t z = cp[cpad(t)] ^ (t + 1 < q ? cp[cpad(q + t)] : 0u);
        for (uint32_t k = 0; k < sh.n_taps; ++k) {
            const uint32_t f = sh.taps[k];
            if (t >= f) z ^= cp[cpad(q + t - f)];
            if (t + 1 < f) z ^= cp[cpad(2 * q + t - f)];
            for (uint32_t k2 = 0; k2 < sh.n_taps; ++k2) {
                const uint32_t gg = sh.taps[k2];
                if (t >= gg && t - gg + 1 < f) z ^= cp[cpad(2 * q + (t - gg) - f)];
            }
        }
        lds[g.zs + bsk_pad(t)] = z;
    }
    __syncthreads();

    // ---- outputs: lane w transposes planes 32w .. 32w + 31 into word w of
    // the 32 outputs and stores them (lanes w adjacent: coalesced per pair)
    uint32_t* ob = reinterpret_cast<uint32_t*>(out + pair0 * qb);
    for (uint32_t w = tid; w < qw; w += nt) {
        uint32_t a[32];
        const uint32_t* zs = lds + g.zs + bsk_pad(32u * w);
#pragma unroll
        for (int i = 0; i < 32; ++i) a[i] = zs[i];
        transpose32(a);
#pragma unroll
        for (uint32_t pp = 0; pp < 32; ++pp)
            if (pp < npw) ob[pp * qw + w] = a[pp];
    }
}

}  // namespace

uint32_t bsk_lds_words(uint32_t q) {
    BskGeom g;
    return bsk_geom(q, &g) ? g.total : 0xffffffffu;
}

hipError_t launch_bsk(const ExtShape& s, const uint8_t* x, const uint8_t* y, uint8_t* out,
                      uint64_t n_pairs, hipStream_t stream) {
    if (n_pairs == 0) return hipSuccess;
    BskGeom g;
    if (!bsk_geom(s.q, &g) || s.n_e == 0 || (uint64_t)s.nbytes * 8 != (uint64_t)s.q * s.n_e)
        return hipErrorInvalidValue;
    if (2 * kBskPairs * g.units > kBskStage * g.threads || g.threads > 448 || g.total * 4 > 65536)
        return hipErrorInvalidValue;
    if (((uintptr_t)x | (uintptr_t)y) & 15u || (uintptr_t)out & 3u) return hipErrorInvalidValue;
    for (uint32_t k = 0; k < s.n_taps; ++k)
        if (s.taps[k] == 0 || 2 * s.taps[k] > s.q) return hipErrorInvalidValue;
    const uint64_t groups = (n_pairs + kBskPairs - 1) / kBskPairs;
    if (groups > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bsk_kernel, dim3((uint32_t)groups), dim3(g.threads), g.total * 4u, stream,
                       x, y, out, n_pairs, s, g);
    return hipGetLastError();
}

}  // namespace qext
