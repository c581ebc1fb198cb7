// SHA-256 (FIPS 180-4) and hashing to F_r for the transcript, on the device.
//
// The paper's random oracles H, H' : {0,1}* -> F_p are instantiated as RFC 9380
// hash_to_field with expand_message_xmd(SHA-256), one element, L = 48 bytes,
// reduced mod r; every use has its own domain-separation tag.  Two forms:
//  * a general byte-streaming hasher for transcript messages (one lane each);
//  * fixed-layout Merkle leaf/node hashing that builds the message words in
//    registers (the 1-byte domain prefix shifts every word by 8 bits).
#pragma once
#include "field.hpp"
#include "tower.hpp"
#include "curve.hpp"

namespace sha {

static constexpr uint32_t K[64] = {
    0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
    0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
    0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
    0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
    0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
    0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
    0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
    0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};

static constexpr uint32_t H0[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                                   0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};

DEV uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

// one compression; w[0..16) is the block as big-endian words
inline NOINL void compress(uint32_t h[8], const uint32_t blk[16]) {
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; i++) w[i] = blk[i];
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
  for (int i = 0; i < 64; i++) {
    uint32_t wi;
    if (i < 16) {
      wi = w[i];
    } else {
      uint32_t w15 = w[(i - 15) & 15], w2 = w[(i - 2) & 15];
      uint32_t s0 = rotr(w15, 7) ^ rotr(w15, 18) ^ (w15 >> 3);
      uint32_t s1 = rotr(w2, 17) ^ rotr(w2, 19) ^ (w2 >> 10);
      wi = w[i & 15] + s0 + w[(i - 7) & 15] + s1;
      w[i & 15] = wi;
    }
    uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    uint32_t ch = (e & f) ^ (~e & g);
    uint32_t t1 = hh + S1 + ch + K[i] + wi;
    uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + S0 + mj;
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

// byte-streaming hasher (buffer kept as 16 big-endian words)
struct Hasher {
  uint32_t h[8];
  uint32_t w[16];
  uint32_t n;        // bytes in the current block
  uint64_t total;    // bytes so far

  HD void init() {
    for (int i = 0; i < 8; i++) h[i] = H0[i];
    for (int i = 0; i < 16; i++) w[i] = 0;
    n = 0;
    total = 0;
  }
  NOINL void byte(uint32_t b) {
    w[n >> 2] |= (b & 0xff) << (24 - 8 * (n & 3));
    n++;
    total++;
    if (n == 64) {
      compress(h, w);
      for (int i = 0; i < 16; i++) w[i] = 0;
      n = 0;
    }
  }
  NOINL void word(uint32_t v) {  // 4 bytes, big-endian
    if ((n & 3) == 0) {
      w[n >> 2] = v;
      n += 4;
      total += 4;
      if (n == 64) {
        compress(h, w);
        for (int i = 0; i < 16; i++) w[i] = 0;
        n = 0;
      }
    } else {
      byte(v >> 24); byte(v >> 16); byte(v >> 8); byte(v);
    }
  }
  HD void u64(uint64_t v) { word((uint32_t)(v >> 32)); word((uint32_t)v); }
  HD void bytes(const uint8_t *p, int len) {
    for (int i = 0; i < len; i++) byte(p[i]);
  }
  HD void str(const char *s) {
    for (; *s; s++) byte((uint8_t)*s);
  }
  // canonical big-endian encoding of a Montgomery-form element
  template <class F> HD void field(const fe &a) {
    fe c = f_from_mont<F>(a);
    for (int i = 7; i >= 0; i--) word(fe_word(c, i));
  }
  HD void g1(const g1_aff &p) { field<FpP>(p.x); field<FpP>(p.y); }
  HD void g2(const g2_aff &p) {
    field<FpP>(p.x.c0); field<FpP>(p.x.c1); field<FpP>(p.y.c0); field<FpP>(p.y.c1);
  }
  HD void gt(const fp12 &f) {
    const fp6 *h6[2] = {&f.c0, &f.c1};
    for (int a = 0; a < 2; a++) {
      const fp2 *q[3] = {&h6[a]->c0, &h6[a]->c1, &h6[a]->c2};
      for (int b = 0; b < 3; b++) { field<FpP>(q[b]->c0); field<FpP>(q[b]->c1); }
    }
  }
  NOINL void final(uint32_t out[8]) {
    uint64_t bits = total * 8;
    byte(0x80);
    total--;  // padding is not message
    while (n != 56) { byte(0); total--; }
    word((uint32_t)(bits >> 32));
    word((uint32_t)bits);
    for (int i = 0; i < 8; i++) out[i] = h[i];
  }
};

DEV int cstrlen(const char *s) {
  int n = 0;
  while (s[n]) n++;
  return n;
}

// expand_message_xmd: start b0 = H(Z_pad || msg || I2OSP(48,2) || 0 || DST || len)
HD inline void xmd_begin(Hasher &hs) {
  hs.init();
  for (int i = 0; i < 16; i++) hs.word(0);  // Z_pad, 64 zero bytes
}

// finish xmd with L = 48 and reduce the 384-bit output mod r; returns Montgomery form
inline NOINL fe xmd_finish_fr(Hasher &hs, const char *dst) {
  int dlen = cstrlen(dst);
  hs.byte(0); hs.byte(48); hs.byte(0);
  hs.str(dst);
  hs.byte((uint32_t)dlen);
  uint32_t b0[8], b1[8], b2[8];
  hs.final(b0);
  Hasher h1;
  h1.init();
  for (int i = 0; i < 8; i++) h1.word(b0[i]);
  h1.byte(1);
  h1.str(dst);
  h1.byte((uint32_t)dlen);
  h1.final(b1);
  Hasher h2;
  h2.init();
  for (int i = 0; i < 8; i++) h2.word(b0[i] ^ b1[i]);
  h2.byte(2);
  h2.str(dst);
  h2.byte((uint32_t)dlen);
  h2.final(b2);
  // uniform = b1 || b2[0..16): hi = b1 words 0..3, lo = b1 words 4..7 || b2 words 0..3
  uint32_t hw[8], lw[8];
  for (int i = 0; i < 4; i++) { hw[i] = b1[3 - i]; hw[4 + i] = 0; }
  for (int i = 0; i < 4; i++) lw[i] = b2[3 - i];
  for (int i = 0; i < 4; i++) lw[4 + i] = b1[7 - i];
  fe hi = fe_from_words(hw), lo = fe_from_words(lw);
  // (hi 2^256 + lo) R mod r = mont(hi, R^3) + mont(lo, R^2)
  return fr_add(fr_mul(hi, fe_const(bn::R_R3)), fr_mul(lo, fe_const(bn::R_R2)));
}

// ---- the same hashes for a message that a workgroup builds together in shared memory:
// the message is kept as big-endian 32-bit words, lanes write its pieces and the padding
// in parallel, and every lane then runs the compression on the same words (plain vector
// code, no per-lane message state).  Coop gives the lane index, the lane count and the
// barrier; the host model runs it as one lane.
struct Coop {
  int lane, n;
#ifdef __HIP_DEVICE_COMPILE__
  __device__ void sync() const { __syncthreads(); }
#else
  HD void sync() const {}
#endif
};

// byte pos of a message held as big-endian words
HD inline void put_byte(uint32_t *w, uint32_t pos, uint32_t v) {
  reinterpret_cast<uint8_t *>(w)[(pos & ~3u) | (3u - (pos & 3u))] = (uint8_t)v;
}

// canonical big-endian words of a Montgomery-form element
template <class F> HD inline void put_words(uint32_t *dst, const fe &a) {
  fe c = f_from_mont<F>(a);
  for (int i = 0; i < 8; i++) dst[i] = fe_word(c, 7 - i);
}

// the same at byte offset pos (any alignment)
template <class F> HD inline void put_field_bytes(uint32_t *w, uint32_t pos, const fe &a) {
  fe c = f_from_mont<F>(a);
  for (int i = 0; i < 32; i++) put_byte(w, pos + i, fe_word(c, 7 - i / 4) >> (24 - 8 * (i & 3)));
}

HD inline void compress_inl(uint32_t h[8], const uint32_t *blk) {
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; i++) w[i] = blk[i];
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
  for (int i = 0; i < 64; i++) {
    uint32_t wi;
    if (i < 16) {
      wi = w[i];
    } else {
      uint32_t w15 = w[(i - 15) & 15], w2 = w[(i - 2) & 15];
      uint32_t s0 = rotr(w15, 7) ^ rotr(w15, 18) ^ (w15 >> 3);
      uint32_t s1 = rotr(w2, 17) ^ rotr(w2, 19) ^ (w2 >> 10);
      wi = w[i & 15] + s0 + w[(i - 7) & 15] + s1;
      w[i & 15] = wi;
    }
    uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    uint32_t ch = (e & f) ^ (~e & g);
    uint32_t t1 = hh + S1 + ch + K[i] + wi;
    uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + S0 + mj;
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

// SHA-256 padding of a len-byte message in w (bytes from len on are overwritten); returns
// the number of blocks.  The caller synchronizes before the blocks are read.
HD inline int pad_coop(const Coop &cp, uint32_t *w, uint32_t len) {
  uint32_t nblk = (len + 8) / 64 + 1, end = 64 * nblk;
  uint64_t bits = (uint64_t)len * 8;
  for (uint32_t p = len + cp.lane; p < end; p += cp.n) {
    uint32_t v = p == len ? 0x80u : p >= end - 8 ? (uint32_t)(bits >> (8 * (end - 1 - p))) & 0xffu : 0u;
    put_byte(w, p, v);
  }
  return (int)nblk;
}

// keeps a value in a vector register: the compression then runs as plain vector code (with
// its rotate, three-input add and xor, and bit-select instructions) instead of alternating
// between the vector and scalar units
#ifdef __HIP_DEVICE_COMPILE__
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}
#else
HD inline uint32_t in_vgpr(uint32_t x) { return x; }
#endif

// digest of the nblk padded blocks in w
HD inline void digest_blocks(const uint32_t *w, int nblk, uint32_t out[8]) {
  uint32_t h[8];
  for (int i = 0; i < 8; i++) h[i] = in_vgpr(H0[i]);
  for (int b = 0; b < nblk; b++) {
    uint32_t blk[16];
#pragma unroll
    for (int i = 0; i < 16; i++) blk[i] = in_vgpr(w[16 * b + i]);
    compress_inl(h, blk);
  }
  for (int i = 0; i < 8; i++) out[i] = h[i];
}

// SHA-256 of the len-byte message in w (room for the padding behind it required); the
// message must be complete (and synchronized) when called; every lane gets the digest
HD inline void sha_coop(const Coop &cp, uint32_t *w, uint32_t len, uint32_t out[8]) {
  int nblk = pad_coop(cp, w, len);
  cp.sync();
  digest_blocks(w, nblk, out);
}

// hash_to_field to F_r (Montgomery form) of the mlen-byte message at byte 64 of w, whose
// first 16 words must be zero (Z_pad of expand_message_xmd, L = 48); w needs room for
// 64 + mlen + the DST suffix + padding (mlen + 64 + 4 + |DST| + 72 bytes), t2 for one
// block; |DST| <= 21.  Same result as Hasher with xmd_begin / xmd_finish_fr.  The message
// must be complete (and synchronized) when called.
HD inline fe xmd_fr_coop(const Coop &cp, uint32_t *w, uint32_t mlen, const char *dst, uint32_t *t2) {
  const uint32_t dlen = (uint32_t)cstrlen(dst), p = 64 + mlen;
  // suffix I2OSP(48, 2) || I2OSP(0, 1) || DST || I2OSP(dlen, 1), then padding
  for (uint32_t i = cp.lane; i < 4 + dlen; i += cp.n)
    put_byte(w, p + i, i == 1 ? 48u : (i == 0 || i == 2) ? 0u : i < 3 + dlen ? (uint32_t)(uint8_t)dst[i - 3] : dlen);
  uint32_t b0[8], b1[8], b2[8];
  sha_coop(cp, w, p + 4 + dlen, b0);
  // b1 = H(b0 || 1 || DST || dlen), b2 = H((b0 xor b1) || 2 || DST || dlen): one block each
  for (int i = 0; i < 8; i++)
    if (i % cp.n == cp.lane) t2[i] = b0[i];
  for (uint32_t i = cp.lane; i < 2 + dlen; i += cp.n)
    put_byte(t2, 32 + i, i == 0 ? 1u : i <= dlen ? (uint32_t)(uint8_t)dst[i - 1] : dlen);
  sha_coop(cp, t2, 34 + dlen, b1);
  cp.sync();
  for (int i = 0; i < 8; i++)
    if (i % cp.n == cp.lane) t2[i] = b0[i] ^ b1[i];
  if (cp.lane == 0) put_byte(t2, 32, 2);
  cp.sync();
  digest_blocks(t2, 1, b2);
  uint32_t hw[8], lw[8];
  for (int i = 0; i < 4; i++) { hw[i] = b1[3 - i]; hw[4 + i] = 0; }
  for (int i = 0; i < 4; i++) lw[i] = b2[3 - i];
  for (int i = 0; i < 4; i++) lw[4 + i] = b1[7 - i];
  fe hi = fe_from_words(hw), lo = fe_from_words(lw);
  return fr_add(fr_mul(hi, fe_const(bn::R_R3)), fr_mul(lo, fe_const(bn::R_R2)));
}

// Merkle leaf SHA-256(0x00 || m_i || C_j): m given as 8 BE words, C as 16 BE words
DEV void merkle_leaf(uint32_t out[8], const uint32_t mw[8], const uint32_t cw[16]) {
  uint32_t x[24];
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = mw[i];
#pragma unroll
  for (int i = 0; i < 16; i++) x[8 + i] = cw[i];
  uint32_t blk[16], h[8];
#pragma unroll
  for (int i = 0; i < 8; i++) h[i] = H0[i];
  // byte stream 0x00 || x: word k = (x[k-1] << 24) | (x[k] >> 8), word 0 = x[0] >> 8
#pragma unroll
  for (int k = 0; k < 16; k++) blk[k] = (k == 0 ? 0u : (x[k - 1] << 24)) | (x[k] >> 8);
  compress(h, blk);
#pragma unroll
  for (int k = 16; k < 24; k++) blk[k - 16] = (x[k - 1] << 24) | (x[k] >> 8);
  blk[8] = (x[23] << 24) | 0x00800000u;  // last message byte then the 0x80 pad byte
#pragma unroll
  for (int k = 9; k < 15; k++) blk[k] = 0;
  blk[15] = 97 * 8;
  compress(h, blk);
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = h[i];
}

// Merkle node SHA-256(0x01 || left || right)
DEV void merkle_node(uint32_t out[8], const uint32_t l[8], const uint32_t r[8]) {
  uint32_t x[16];
#pragma unroll
  for (int i = 0; i < 8; i++) { x[i] = l[i]; x[8 + i] = r[i]; }
  uint32_t blk[16], h[8];
#pragma unroll
  for (int i = 0; i < 8; i++) h[i] = H0[i];
#pragma unroll
  for (int k = 0; k < 16; k++) blk[k] = (k == 0 ? 0x01000000u : (x[k - 1] << 24)) | (x[k] >> 8);
  compress(h, blk);
  blk[0] = (x[15] << 24) | 0x00800000u;
#pragma unroll
  for (int k = 1; k < 15; k++) blk[k] = 0;
  blk[15] = 65 * 8;
  compress(h, blk);
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = h[i];
}

}  // namespace sha
