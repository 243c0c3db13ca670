// SHA-256 (FIPS 180-4) for the cryptographic layout streams: counter-mode
// words SHA-256(seed_le64 || tag_le32 || idx_le32 || block_le64), each
// 32-byte digest giving four little-endian 64-bit words.
//
// The round constants and the initial hash value are derived here from their
// definition instead of being tabulated: the first 32 bits of the fractional
// parts of the cube roots of the first 64 primes, and of the square roots of
// the first 8 primes, each settled by an exact integer comparison.

#include <cmath>
#include <cstring>

#include "cloak_internal.hpp"

namespace cloak {
namespace {

struct Constants {
  uint32_t k[64];
  uint32_t h0[8];
  Constants() {
    int primes[64];
    int n = 0;
    for (int c = 2; n < 64; ++c) {
      bool prime = true;
      for (int d = 2; d * d <= c; ++d)
        if (c % d == 0) prime = false;
      if (prime) primes[n++] = c;
    }
    using u128 = unsigned __int128;
    for (int i = 0; i < 64; ++i) {
      // x = floor(cbrt(p) * 2^32): the largest x with x^3 <= p * 2^96
      const u128 target = u128(uint64_t(primes[i])) << 96;
      uint64_t x = uint64_t(std::cbrt(double(primes[i])) * 4294967296.0);
      while (u128(x) * x * x > target) --x;
      while (u128(x + 1) * (x + 1) * (x + 1) <= target) ++x;
      k[i] = uint32_t(x);  // the low 32 bits are the fractional part
    }
    for (int i = 0; i < 8; ++i) {
      const u128 target = u128(uint64_t(primes[i])) << 64;
      uint64_t x = uint64_t(std::sqrt(double(primes[i])) * 4294967296.0);
      while (u128(x) * x > target) --x;
      while (u128(x + 1) * (x + 1) <= target) ++x;
      h0[i] = uint32_t(x);
    }
  }
};

const Constants& constants() {
  static const Constants c;
  return c;
}

inline uint32_t rotr(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }

void compress(uint32_t h[8], const uint8_t block[64]) {
  const Constants& c = constants();
  uint32_t w[64];
  for (int t = 0; t < 16; ++t)
    w[t] = uint32_t(block[4 * t]) << 24 | uint32_t(block[4 * t + 1]) << 16 | uint32_t(block[4 * t + 2]) << 8 |
           uint32_t(block[4 * t + 3]);
  for (int t = 16; t < 64; ++t) {
    const uint32_t s0 = rotr(w[t - 15], 7) ^ rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
    const uint32_t s1 = rotr(w[t - 2], 17) ^ rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
    w[t] = w[t - 16] + s0 + w[t - 7] + s1;
  }
  uint32_t a = h[0], b = h[1], cc = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
  for (int t = 0; t < 64; ++t) {
    const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = hh + S1 + ch + c.k[t] + w[t];
    const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    const uint32_t maj = (a & b) ^ (a & cc) ^ (b & cc);
    const uint32_t t2 = S0 + maj;
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = cc;
    cc = b;
    b = a;
    a = t1 + t2;
  }
  h[0] += a; h[1] += b; h[2] += cc; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

}  // namespace

void sha256(const uint8_t* msg, size_t len, uint8_t out[32]) {
  uint32_t h[8];
  std::memcpy(h, constants().h0, sizeof h);
  uint8_t block[64];
  size_t off = 0;
  for (; off + 64 <= len; off += 64) compress(h, msg + off);
  // padding: 0x80, zeros, message length in bits (big-endian), one or two blocks
  const size_t rest = len - off;
  std::memset(block, 0, 64);
  std::memcpy(block, msg + off, rest);
  block[rest] = 0x80;
  if (rest >= 56) {
    compress(h, block);
    std::memset(block, 0, 64);
  }
  const uint64_t bits = uint64_t(len) * 8;
  for (int i = 0; i < 8; ++i) block[63 - i] = uint8_t(bits >> (8 * i));
  compress(h, block);
  for (int i = 0; i < 8; ++i) {
    out[4 * i] = uint8_t(h[i] >> 24);
    out[4 * i + 1] = uint8_t(h[i] >> 16);
    out[4 * i + 2] = uint8_t(h[i] >> 8);
    out[4 * i + 3] = uint8_t(h[i]);
  }
}

uint64_t Sha256Ctr::next() {
  if (j % 4 == 0) {
    uint8_t msg[24];
    const uint64_t blk = j / 4;
    std::memcpy(msg, prefix, 16);
    for (int i = 0; i < 8; ++i) msg[16 + i] = uint8_t(blk >> (8 * i));
    sha256(msg, sizeof msg, digest);
  }
  uint64_t w = 0;
  for (int i = 7; i >= 0; --i) w = (w << 8) | digest[8 * (j % 4) + i];
  ++j;
  return w;
}

Sha256Ctr sha256_substream(uint64_t seed, uint32_t tag, uint32_t idx) {
  Sha256Ctr g;
  for (int i = 0; i < 8; ++i) g.prefix[i] = uint8_t(seed >> (8 * i));
  for (int i = 0; i < 4; ++i) g.prefix[8 + i] = uint8_t(tag >> (8 * i));
  for (int i = 0; i < 4; ++i) g.prefix[12 + i] = uint8_t(idx >> (8 * i));
  return g;
}

}  // namespace cloak
