// Occupancy summary of the buckets: which buckets hold at least one key.
//
// Successor and range queries continue into the next bucket that holds a key,
// and predecessor queries into the previous one (Section 2.1 operations; the
// paper's successor experiments, Section 6.5, run after rounds of deletes).
// After clustered deletes thousands of consecutive buckets can be empty, so a
// walk over bucket headers would be linear in the gap.  Three bit levels make
// the search logarithmic in base 64:
//   level 0: bit b       = bucket b is not empty
//   level 1: bit w       = level-0 word w is not zero  (64 buckets per bit)
//   level 2: bit v       = level-1 word v is not zero  (4096 buckets per bit)
// A search reads at most one word per level on the way up and down, plus
// level-2 words one after another (each covers 262144 buckets).
//
// The update kernels keep it current: an insert that fills an empty bucket
// sets its bit, a delete that empties a bucket clears it, and a word that
// becomes non-zero or zero carries the change one level up (the returned old
// word tells which call did it).  Inserts and deletes never run in the same
// kernel, so sets and clears never race with each other.  The kernels that
// build and check the summary are in flix_build.hpp.
#pragma once

#include "flix_device.hpp"

namespace flix {

struct OccLevels {
  u64* w0;   // [ceil(nb / 64)]
  u64* w1;   // [ceil(nb / 4096)]
  u64* w2;   // [ceil(nb / 262144)]
};

__host__ __device__ inline u64 occ_words0(u64 nb) { return (nb + 63) / 64; }
__host__ __device__ inline u64 occ_words1(u64 nb) { return (occ_words0(nb) + 63) / 64; }
__host__ __device__ inline u64 occ_words2(u64 nb) { return (occ_words1(nb) + 63) / 64; }
__host__ __device__ inline u64 occ_words(u64 nb) {
  return occ_words0(nb) + occ_words1(nb) + occ_words2(nb);
}

// The three levels of a summary laid out one after another from w0 (as the
// store allocates them), for nb buckets.
__host__ __device__ inline OccLevels occ_levels(u64* w0, u64 nb) {
  OccLevels o;
  o.w0 = w0;
  o.w1 = w0 + occ_words0(nb);
  o.w2 = o.w1 + occ_words1(nb);
  return o;
}

__host__ __device__ __forceinline__ u32 ctz64(u64 x) { return (u32)__builtin_ctzll(x); }
__host__ __device__ __forceinline__ u32 top64(u64 x) { return 63u - (u32)__builtin_clzll(x); }

// Bucket b now holds keys (it was empty).
__device__ __forceinline__ void occ_set(const OccLevels& o, u32 b) {
  const u64 bit0 = 1ull << (b & 63);
  const u64 old0 = atomicOr((unsigned long long*)&o.w0[b >> 6], (unsigned long long)bit0);
  if (old0 != 0) return;
  const u32 i1 = b >> 6;
  const u64 bit1 = 1ull << (i1 & 63);
  const u64 old1 = atomicOr((unsigned long long*)&o.w1[i1 >> 6], (unsigned long long)bit1);
  if (old1 != 0) return;
  const u32 i2 = i1 >> 6;
  atomicOr((unsigned long long*)&o.w2[i2 >> 6], (unsigned long long)(1ull << (i2 & 63)));
}

// Bucket b is now empty (it held keys).
__device__ __forceinline__ void occ_clear(const OccLevels& o, u32 b) {
  const u64 bit0 = 1ull << (b & 63);
  const u64 old0 = atomicAnd((unsigned long long*)&o.w0[b >> 6], (unsigned long long)~bit0);
  if (old0 != bit0) return;   // other buckets of the word still hold keys (or it was clear)
  const u32 i1 = b >> 6;
  const u64 bit1 = 1ull << (i1 & 63);
  const u64 old1 = atomicAnd((unsigned long long*)&o.w1[i1 >> 6], (unsigned long long)~bit1);
  if (old1 != bit1) return;
  const u32 i2 = i1 >> 6;
  atomicAnd((unsigned long long*)&o.w2[i2 >> 6], (unsigned long long)~(1ull << (i2 & 63)));
}

// First bucket after b that holds a key, or nb when none exists.
__host__ __device__ inline u32 occ_next(const OccLevels& o, u32 nb, u32 b) {
  const u64 n0 = occ_words0(nb), n1 = occ_words1(nb), n2 = occ_words2(nb);
  const u64 i = (u64)b + 1;
  if (i >= nb) return nb;
  const u64 w0i = i >> 6;
  u64 m = o.w0[w0i] & (~0ull << (i & 63));
  if (m) return (u32)((w0i << 6) + ctz64(m));
  // later words of the same level-1 word
  const u64 j = w0i + 1;
  if (j >= n0) return nb;
  const u64 w1i = j >> 6;
  m = o.w1[w1i] & (~0ull << (j & 63));
  u64 w0f;
  if (m) {
    w0f = (w1i << 6) + ctz64(m);
  } else {
    // later level-1 words, through level 2
    const u64 k = w1i + 1;
    if (k >= n1) return nb;
    u64 w2i = k >> 6;
    m = o.w2[w2i] & (~0ull << (k & 63));
    while (!m) {
      if (++w2i >= n2) return nb;
      m = o.w2[w2i];
    }
    const u64 w1f = (w2i << 6) + ctz64(m);
    const u64 mm = o.w1[w1f];
    if (!mm) return nb;   // levels disagree: never on a consistent summary
    w0f = (w1f << 6) + ctz64(mm);
  }
  const u64 z = o.w0[w0f];
  if (!z) return nb;
  const u64 r = (w0f << 6) + ctz64(z);
  return r < nb ? (u32)r : nb;
}

// Last bucket before b that holds a key, or kNil when none exists.
__host__ __device__ inline u32 occ_prev(const OccLevels& o, u32 b) {
  if (b == 0) return kNil;
  const u64 i = (u64)b - 1;
  const u64 w0i = i >> 6;
  u64 m = o.w0[w0i] & (~0ull >> (63 - (i & 63)));
  if (m) return (u32)((w0i << 6) + top64(m));
  if (w0i == 0) return kNil;
  const u64 j = w0i - 1;
  const u64 w1i = j >> 6;
  m = o.w1[w1i] & (~0ull >> (63 - (j & 63)));
  u64 w0f;
  if (m) {
    w0f = (w1i << 6) + top64(m);
  } else {
    if (w1i == 0) return kNil;
    const u64 k = w1i - 1;
    u64 w2i = k >> 6;
    m = o.w2[w2i] & (~0ull >> (63 - (k & 63)));
    while (!m) {
      if (w2i == 0) return kNil;
      m = o.w2[--w2i];
    }
    const u64 w1f = (w2i << 6) + top64(m);
    const u64 mm = o.w1[w1f];
    if (!mm) return kNil;
    w0f = (w1f << 6) + top64(mm);
  }
  const u64 z = o.w0[w0f];
  if (!z) return kNil;
  return (u32)((w0f << 6) + top64(z));
}

}  // namespace flix
