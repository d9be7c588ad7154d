// Split stream: one lane per resampled split.
//
// Split b draws its nx members out of the n = nx + ny pooled items (X rows,
// then Y rows) by selection sampling (Knuth, TAOCP vol. 2, 3.4.2, Algorithm S):
// item t joins x* with probability need/(n - t), decided in integers as
// floor(u_t (n - t) / 2^64) < need, where u_t is a 64-bit Philox4x32-10 draw
// (Salmon et al., SC'11) with key (seed_lo, seed_hi) and counter
// (t/2, b_lo, b_hi, 0); even t uses output words (0, 1), odd t words (2, 3),
// low word first.  Once need is 0 (or equals the items left) the outcome is
// fixed and no draw is needed.  This replaces Alg. 2's SampleWithoutReplacement;
// the statistic only depends on which items form x*.
#include "common.h"

namespace et {

__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

struct SplitDraw {
  uint32_t k0, k1, b_lo, b_hi;
  int64_t n, need, t;
  uint4 rnd;
  uint32_t pair;  // counter word 0 of the cached Philox block (0xFFFFFFFF: none)

  __device__ SplitDraw(uint64_t seed, uint64_t b, int64_t nx, int64_t ny)
      : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), b_lo((uint32_t)b),
        b_hi((uint32_t)(b >> 32)), n(nx + ny), need(nx), t(0), rnd(make_uint4(0, 0, 0, 0)),
        pair(0xFFFFFFFFu) {}

  // Decide the next pooled item (items are visited in order t = 0, 1, ...).
  __device__ uint32_t next() {
    const int64_t m = n - t;
    uint32_t take;
    if (need == 0) {
      take = 0;
    } else if (need == m) {
      take = 1;
    } else {
      const uint32_t c = (uint32_t)(t >> 1);
      if (pair != c) {
        rnd = philox4x32_10(make_uint4(c, b_lo, b_hi, 0u), k0, k1);
        pair = c;
      }
      const uint32_t lo = (t & 1) ? rnd.z : rnd.x;
      const uint32_t hi = (t & 1) ? rnd.w : rnd.y;
      const uint64_t mm = (uint64_t)m;
      const uint64_t p_lo = (uint64_t)lo * mm;
      const uint64_t p_hi = (uint64_t)hi * mm;
      const uint64_t v = (p_hi + (p_lo >> 32)) >> 32;  // floor(u * m / 2^64)
      take = v < (uint64_t)need ? 1u : 0u;
    }
    need -= take;
    ++t;
    return take;
  }
};

// Internal layout Z[w][col]: columns 0..B-1 drawn splits, B the identity split,
// the rest zero; words cover padded pooled positions (X tiles, then Y tiles).
__global__ void __launch_bounds__(256) k_member(const TestDesc* __restrict__ descs,
                                                const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc& d = descs[ti];
  const int64_t col = (blockIdx.x - offs[ti]) * 256 + threadIdx.x;
  if (col >= d.B_pad) return;
  uint32_t* Z = d.Z;
  const int xw = d.tx * TILE_WORDS, yw = d.ty * TILE_WORDS;
  if (col >= d.B) {
    const bool ident = col == d.B;
    for (int w = 0; w < xw; ++w) {
      uint32_t word = 0;
      if (ident) {
        const int lo = w * 32;
        const int cnt = d.nx - lo;
        word = cnt >= 32 ? 0xFFFFFFFFu : (cnt > 0 ? ((1u << cnt) - 1u) : 0u);
      }
      Z[(int64_t)w * d.B_pad + col] = word;
    }
    for (int w = 0; w < yw; ++w) Z[(int64_t)(xw + w) * d.B_pad + col] = 0u;
    return;
  }
  SplitDraw s(d.seed, (uint64_t)col, d.nx, d.ny);
  for (int w = 0; w < xw; ++w) {
    uint32_t word = 0;
    for (int bit = 0; bit < 32; ++bit)
      if (w * 32 + bit < d.nx) word |= s.next() << bit;
    Z[(int64_t)w * d.B_pad + col] = word;
  }
  for (int w = 0; w < yw; ++w) {
    uint32_t word = 0;
    for (int bit = 0; bit < 32; ++bit)
      if (w * 32 + bit < d.ny) word |= s.next() << bit;
    Z[(int64_t)(xw + w) * d.B_pad + col] = word;
  }
}

// Public layout: words[(b - b0) * W + t / 32], bit t % 32, W = ceil(n / 32).
__global__ void __launch_bounds__(256) k_member_public(int64_t nx, int64_t ny, uint64_t seed,
                                                       int64_t b0, int64_t count,
                                                       uint32_t* __restrict__ words) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= count) return;
  const int64_t n = nx + ny, W = (n + 31) / 32;
  SplitDraw s(seed, (uint64_t)(b0 + q), nx, ny);
  uint32_t* out = words + q * W;
  for (int64_t w = 0; w < W; ++w) {
    uint32_t word = 0;
    for (int bit = 0; bit < 32; ++bit)
      if (w * 32 + bit < n) word |= s.next() << bit;
    out[w] = word;
  }
}

void launch_member(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_member, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}
void launch_member_public(int64_t nx, int64_t ny, uint64_t seed, int64_t b0, int64_t count,
                          uint32_t* words, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_member_public, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, nx,
                     ny, seed, b0, count, words);
}

}  // namespace et
