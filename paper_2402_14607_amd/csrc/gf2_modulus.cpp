// gf2_modulus.cpp -- the library's modulus convention for F_{2^m}.
//
// The paper fixes the field F_{2^q} (Def. 3.2) but not its representation.
// The library uses the polynomial basis modulo the lowest-weight irreducible
// P of degree m, ties broken by the lexicographically smallest exponents:
// a trinomial t^m + t^a + 1 with least a if one exists, otherwise a
// pentanomial t^m + t^a + t^b + t^c + 1 with least a, then b, then c.
//
// Irreducibility is decided by Rabin's test: P of degree m is irreducible
// iff t^(2^m) = t mod P and gcd(t^(2^(m/r)) - t, P) = 1 for each prime r | m.
// Candidates are first sieved by divisibility by the irreducible polynomials
// of degree <= 12, and trinomials are skipped when m = 0 mod 8 (Swan 1962:
// t^m + t^a + 1 then has an even number of irreducible factors).
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gf2_modulus.h"

namespace qext {
namespace {

using Poly = std::vector<uint64_t>;

// Insert a zero between consecutive bits of a 32-bit value (squaring in
// characteristic 2 sends t^i to t^(2i)).
inline uint64_t interleave_zeros(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

int degree(const Poly& a) {
    for (size_t i = a.size(); i-- > 0;)
        if (a[i]) return (int)(i * 64) + 63 - __builtin_clzll(a[i]);
    return -1;
}

struct SparseModulus {
    uint32_t m;
    std::vector<uint32_t> low;  // exponents below m (including 0)
};

// Fold the part of `a` of degree >= m down with t^m = sum_{e in low} t^e,
// whole words at a time: H = a >> m is cleared from `a` and H * t^e added
// for every low exponent e; repeated while the sum still reaches degree m
// (twice for moduli whose taps lie far below m).
void reduce(Poly& a, const SparseModulus& P, Poly& hi) {
    const uint32_t m = P.m;
    const size_t n = a.size();
    const uint32_t ws = m >> 6, bs = m & 63;
    for (;;) {
        const int d = degree(a);
        if (d < (int)m) return;
        const size_t hw = (size_t)(d - (int)m) / 64 + 1;  // words of H
        for (size_t i = 0; i < hw; ++i) {
            const size_t s = ws + i;
            uint64_t v = a[s] >> bs;
            if (bs && s + 1 < n) v |= a[s + 1] << (64 - bs);
            hi[i] = v;
        }
        // clear bits >= m
        if (bs) a[ws] &= (1ull << bs) - 1;
        for (size_t i = ws + (bs ? 1 : 0); i < n; ++i) a[i] = 0;
        for (uint32_t e : P.low) {
            const uint32_t ew = e >> 6, eb = e & 63;
            if (eb == 0) {
                for (size_t i = 0; i < hw; ++i) a[ew + i] ^= hi[i];
            } else {
                for (size_t i = 0; i < hw; ++i) {
                    a[ew + i] ^= hi[i] << eb;
                    a[ew + i + 1] ^= hi[i] >> (64 - eb);
                }
            }
        }
    }
}

// a <- a^2 mod P (deg a < m); tmp and hi hold 2 * words(m) + 2 words.
void square_mod(Poly& a, const SparseModulus& P, Poly& tmp, Poly& hi) {
    const size_t nw = (P.m + 63) / 64;
    for (size_t i = 0; i < nw; ++i) {
        tmp[2 * i] = interleave_zeros((uint32_t)a[i]);
        tmp[2 * i + 1] = interleave_zeros((uint32_t)(a[i] >> 32));
    }
    std::fill(tmp.begin() + 2 * nw, tmp.end(), 0);
    reduce(tmp, P, hi);
    std::copy(tmp.begin(), tmp.begin() + nw, a.begin());
}

// Binary (Stein) gcd over GF(2)[t] for two polynomials, returns degree of
// gcd (0 means coprime).  a, b are consumed.
int gcd_degree(Poly a, Poly b) {
    auto shift_out_t = [](Poly& p) {
        // divide by the largest power of t dividing p (p nonzero)
        size_t z = 0;
        while (p[z] == 0) ++z;
        const int tz = __builtin_ctzll(p[z]);
        const size_t n = p.size();
        for (size_t i = 0; i < n; ++i) {
            const size_t s = i + z;
            uint64_t v = s < n ? p[s] >> tz : 0;
            if (tz && s + 1 < n) v |= p[s + 1] << (64 - tz);
            p[i] = v;
        }
    };
    int da = degree(a), db = degree(b);
    if (da < 0) return db;
    if (db < 0) return da;
    // The common factor t^k is not tracked: callers pass b with constant
    // term 1 (the modulus), so t never divides the gcd.
    shift_out_t(a);
    shift_out_t(b);
    for (;;) {
        da = degree(a);
        db = degree(b);
        if (da < db) {
            std::swap(a, b);
            std::swap(da, db);
        }
        if (db == 0) return 0;  // b == 1
        for (size_t i = 0; i < a.size(); ++i) a[i] ^= b[i];
        if (degree(a) < 0) return db;
        shift_out_t(a);
    }
}

std::vector<uint32_t> prime_factors(uint32_t m) {
    std::vector<uint32_t> r;
    for (uint32_t p = 2; p * p <= m; ++p)
        if (m % p == 0) {
            r.push_back(p);
            while (m % p == 0) m /= p;
        }
    if (m > 1) r.push_back(m);
    return r;
}

// Rabin's test along one squaring chain t, t^2, t^4, ... mod P: the values
// t^(2^(m/r)) for the primes r | m are kept on the way to t^(2^m), and their
// gcds with P are taken only when t^(2^m) = t holds (nearly every reducible
// candidate fails that first).
bool rabin(const SparseModulus& P) {
    const uint32_t m = P.m;
    if (m == 1) return true;
    const size_t nw = (m + 63) / 64 + 1;
    Poly tmp(2 * nw + 2), hi(2 * nw + 2);
    Poly full(nw, 0);
    full[m >> 6] |= 1ull << (m & 63);
    for (uint32_t e : P.low) full[e >> 6] ^= 1ull << (e & 63);
    const std::vector<uint32_t> primes = prime_factors(m);
    std::vector<Poly> kept(primes.size());
    Poly h(nw, 0);
    h[0] = 2;  // t
    for (uint32_t i = 1; i <= m; ++i) {
        square_mod(h, P, tmp, hi);
        for (size_t k = 0; k < primes.size(); ++k)
            if (i == m / primes[k]) kept[k] = h;
    }
    h[0] ^= 2;
    if (degree(h) >= 0) return false;
    for (Poly& g : kept) {
        g[0] ^= 2;  // t^(2^(m/r)) - t
        if (degree(g) < 0) return false;
        if (gcd_degree(g, full) != 0) return false;
    }
    return true;
}

// ---- sieve: irreducible polynomials of degree <= 12 and powers of t ------
struct SmallIrr {
    uint32_t f;
    int deg;
    std::vector<uint16_t> pw;  // t^k mod f for k = 0 .. ord-1 (ord = order of t)
};

int small_degree(uint32_t v) { return v ? 31 - __builtin_clz(v) : -1; }

uint32_t times_t_mod(uint32_t v, uint32_t f, int d) {
    v <<= 1;
    if ((v >> d) & 1) v ^= f;
    return v;
}

const std::vector<SmallIrr>& small_irreducibles() {
    static std::vector<SmallIrr> list;
    static std::once_flag once;
    std::call_once(once, [] {
        const int maxdeg = 12;
        // sieve of Eratosthenes on polynomials: mark every product f*g
        const uint32_t lim = 1u << (maxdeg + 1);
        std::vector<uint8_t> composite(lim, 0);
        auto clmul = [](uint32_t a, uint32_t b) {
            uint32_t r = 0;
            for (int i = 0; b >> i; ++i)
                if ((b >> i) & 1) r ^= a << i;
            return r;
        };
        for (uint32_t a = 2; a < lim; ++a)
            for (uint32_t b = 2; b <= a; ++b) {
                if (small_degree(a) + small_degree(b) > maxdeg) break;
                composite[clmul(a, b)] = 1;
            }
        for (uint32_t f = 2; f < lim; ++f) {
            if (composite[f]) continue;
            SmallIrr s;
            s.f = f;
            s.deg = small_degree(f);
            if (!(f & 1)) {  // f = t: t^k mod t = 0 for k >= 1
                s.pw = {1};
                list.push_back(s);
                continue;
            }
            uint32_t v = 1;
            do {
                s.pw.push_back((uint16_t)v);
                v = times_t_mod(v, f, s.deg);
            } while (v != 1);
            list.push_back(std::move(s));
        }
    });
    return list;
}

uint32_t t_pow_mod_small(const SmallIrr& s, uint32_t k) {
    if (!(s.f & 1)) return k == 0 ? 1u : 0u;
    return s.pw[k % s.pw.size()];
}

bool sieved_out(uint32_t m, const std::vector<uint32_t>& low) {
    for (const SmallIrr& s : small_irreducibles()) {
        if ((uint32_t)s.deg >= m) break;
        uint32_t v = t_pow_mod_small(s, m);
        for (uint32_t e : low) v ^= t_pow_mod_small(s, e);
        if (v == 0) return true;
    }
    return false;
}

}  // namespace

bool modulus_is_irreducible(uint32_t m, const uint32_t* taps, uint32_t n_taps) {
    SparseModulus P{m, {0}};
    for (uint32_t k = 0; k < n_taps; ++k) P.low.push_back(taps[k]);
    return rabin(P);
}

namespace {

// Candidates in the convention's order (trinomials when m % 8 != 0, then
// pentanomials by a, b, c), sieved serially; the survivors go through
// Rabin's test in batches on worker threads, and the first irreducible one
// in order wins.
bool search_ordered(uint32_t m, std::vector<uint32_t>* taps) {
    const unsigned hw = std::thread::hardware_concurrency();
    const unsigned nthr = std::max(1u, std::min(hw ? hw : 1u, 16u));
    std::vector<std::vector<uint32_t>> batch;
    const size_t batch_cap = 4 * nthr;
    auto run_batch = [&]() -> bool {
        std::vector<uint8_t> ok(batch.size(), 0);
        std::atomic<size_t> next{0};
        auto work = [&]() {
            for (;;) {
                const size_t i = next.fetch_add(1);
                if (i >= batch.size()) return;
                SparseModulus P{m, batch[i]};
                ok[i] = rabin(P) ? 1 : 0;
            }
        };
        std::vector<std::thread> th;
        for (unsigned t = 1; t < nthr && t < batch.size(); ++t) th.emplace_back(work);
        work();
        for (auto& t : th) t.join();
        for (size_t i = 0; i < batch.size(); ++i)
            if (ok[i]) {
                taps->assign(batch[i].begin(), batch[i].end() - 1);  // drop the 0
                return true;
            }
        batch.clear();
        return false;
    };
    auto offer = [&](std::vector<uint32_t> low) -> bool {
        if (sieved_out(m, low)) return false;
        batch.push_back(std::move(low));
        return batch.size() >= batch_cap && run_batch();
    };
    if (m % 8 != 0) {
        for (uint32_t a = 1; 2 * a <= m; ++a)
            if (offer({a, 0})) return true;
        if (!batch.empty() && run_batch()) return true;
    }
    for (uint32_t a = 3; a < m; ++a)
        for (uint32_t b = 2; b < a; ++b)
            for (uint32_t c = 1; c < b; ++c)
                if (offer({a, b, c, 0})) return true;
    return !batch.empty() && run_batch();
}

}  // namespace

bool search_modulus(uint32_t m, std::vector<uint32_t>* taps) {
    if (m < 2) return false;
    return search_ordered(m, taps);
}

// Conventional modulus of degree m: the library's table when it has the
// degree, else a search (cached) for m up to kSearchLimit.
bool default_modulus(uint32_t m, std::vector<uint32_t>* taps) {
    static const struct {
        uint32_t m, n, t[3];
    } table[] = {
#ifndef QEXT_NO_TABLE
#include "moduli_table.inc"
#endif
        {0, 0, {0, 0, 0}},  // end
    };
    for (const auto& r : table)
        if (r.m && r.m == m) {
            taps->assign(r.t, r.t + r.n);
            return true;
        }
    if (m > kSearchLimit) return false;
    static std::mutex mu;
    static std::unordered_map<uint32_t, std::vector<uint32_t>> cache;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(m);
        if (it != cache.end()) {
            *taps = it->second;
            return true;
        }
    }
    std::vector<uint32_t> found;
    if (!search_modulus(m, &found)) return false;
    std::lock_guard<std::mutex> g(mu);
    cache[m] = found;
    *taps = found;
    return true;
}

}  // namespace qext
