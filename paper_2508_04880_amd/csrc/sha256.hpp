// sha256.hpp -- SHA-256 as specified in FIPS 180-4 (Secure Hash Standard),
// streaming.  The 64 round constants and the initial hash value are formed
// from their definition in the standard: the first 32 bits of the fractional
// parts of the cube roots of the first 64 primes, and of the square roots of
// the first 8.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

namespace tusq {

class Sha256 {
public:
    Sha256() {
        const Tables &t = tables();
        for (int i = 0; i < 8; ++i) h_[i] = t.h0[i];
    }

    void update(const void *data, size_t len) {
        const uint8_t *p = static_cast<const uint8_t *>(data);
        total_ += len;
        while (len) {
            const size_t take = len < 64 - fill_ ? len : 64 - fill_;
            for (size_t i = 0; i < take; ++i) block_[fill_ + i] = p[i];
            fill_ += take;
            p += take;
            len -= take;
            if (fill_ == 64) {
                compress();
                fill_ = 0;
            }
        }
    }

    // Pads (a one bit, zeros, the 64-bit big-endian message length in bits)
    // and writes the digest big-endian.
    void finish(uint8_t out[32]) {
        const uint64_t bits = total_ * 8;
        block_[fill_++] = 0x80;
        if (fill_ > 56) {
            while (fill_ < 64) block_[fill_++] = 0;
            compress();
            fill_ = 0;
        }
        while (fill_ < 56) block_[fill_++] = 0;
        for (int i = 0; i < 8; ++i) block_[56 + i] = static_cast<uint8_t>(bits >> (56 - 8 * i));
        compress();
        fill_ = 0;
        for (int i = 0; i < 8; ++i)
            for (int b = 0; b < 4; ++b) out[4 * i + b] = static_cast<uint8_t>(h_[i] >> (24 - 8 * b));
    }

private:
    struct Tables {
        uint32_t k[64];
        uint32_t h0[8];
    };

    // first 32 fractional bits of r (r > 0)
    static uint32_t frac32(long double r) {
        const long double f = r - std::floor(r);
        return static_cast<uint32_t>(std::floor(std::ldexp(f, 32)));
    }

    static const Tables &tables() {
        static const Tables t = [] {
            Tables x{};
            int found = 0;
            for (int cand = 2; found < 64; ++cand) {
                bool prime = true;
                for (int d = 2; d * d <= cand; ++d)
                    if (cand % d == 0) { prime = false; break; }
                if (!prime) continue;
                x.k[found] = frac32(std::cbrt(static_cast<long double>(cand)));
                if (found < 8) x.h0[found] = frac32(std::sqrt(static_cast<long double>(cand)));
                ++found;
            }
            return x;
        }();
        return t;
    }

    static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

    void compress() {
        const Tables &t = tables();
        uint32_t w[64];
        for (int i = 0; i < 16; ++i)
            w[i] = (uint32_t(block_[4 * i]) << 24) | (uint32_t(block_[4 * i + 1]) << 16) |
                   (uint32_t(block_[4 * i + 2]) << 8) | uint32_t(block_[4 * i + 3]);
        for (int i = 16; i < 64; ++i) {
            const uint32_t s0 = rotr(w[i - 15], 7) ^ rotr(w[i - 15], 18) ^ (w[i - 15] >> 3);
            const uint32_t s1 = rotr(w[i - 2], 17) ^ rotr(w[i - 2], 19) ^ (w[i - 2] >> 10);
            w[i] = w[i - 16] + s0 + w[i - 7] + s1;
        }
        uint32_t a = h_[0], b = h_[1], c = h_[2], d = h_[3], e = h_[4], f = h_[5], g = h_[6],
                 h = h_[7];
        for (int i = 0; i < 64; ++i) {
            const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
            const uint32_t ch = (e & f) ^ (~e & g);
            const uint32_t t1 = h + S1 + ch + t.k[i] + w[i];
            const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
            const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
            const uint32_t t2 = S0 + maj;
            h = g;
            g = f;
            f = e;
            e = d + t1;
            d = c;
            c = b;
            b = a;
            a = t1 + t2;
        }
        h_[0] += a; h_[1] += b; h_[2] += c; h_[3] += d;
        h_[4] += e; h_[5] += f; h_[6] += g; h_[7] += h;
    }

    uint32_t h_[8];
    uint8_t block_[64] = {};
    size_t fill_ = 0;
    uint64_t total_ = 0;
};

}  // namespace tusq
