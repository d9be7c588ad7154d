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
//
// One workgroup serves MSPL consecutive split columns and walks the pooled
// tiles in order (one tile = 128 padded positions = 4 words).  The scaled draws
// v_t = floor(u_t (n - t) / 2^64) do not depend on the running count, so waves 1..3
// produce the next tile's draws into LDS while wave 0 runs the selection scan (one
// lane per split) over the current one.  Positions without an item (tile padding)
// hold v = 0xFFFFFFFF, which is never below need (< 2^31), so the scan is the same
// branch-free step for every position and writes whole words.
__device__ inline uint32_t scaled_draw(uint32_t lo, uint32_t hi, uint32_t m) {
  const uint64_t p_lo = (uint64_t)lo * m, p_hi = (uint64_t)hi * m;
  return (uint32_t)((p_hi + (p_lo >> 32)) >> 32);  // floor(u * m / 2^64), u = hi:lo
}

// MSPL is MEMBER_SPLITS, or MEMBER_SPLITS_WIDE for a launch with more workgroups than the
// chip holds at once: there the stream is bound by vector-ALU cycles, and a wider
// workgroup keeps twice as many of the scanning wave's lanes busy.
template <int MSPL>
__global__ void __launch_bounds__(MTHREADS) k_member(const TestDesc* __restrict__ descs,
                                                const int64_t* __restrict__ offs, int ntests) {
  __shared__ uint32_t V[2][TILE][MSPL];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t col0 = (blockIdx.x - offs[ti]) * MSPL;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t n = (int64_t)d.nx + d.ny;
  const int xw = d.tx * TILE_WORDS, nwords = d.nt * TILE_WORDS;
  uint32_t* Z = d.Z;
  const int64_t BP = d.B_pad;
  // non-drawn columns: the identity split (column B) and zero padding
  if (col0 + MSPL > d.B) {
    for (int e = tid; e < nwords * MSPL; e += MTHREADS) {
      const int w = e / MSPL;
      const int64_t c = col0 + e % MSPL;
      if (c < d.B) continue;
      uint32_t v = 0;
      if (c == d.B && w < xw) {
        const int64_t cnt = d.nx - (int64_t)w * 32;
        v = cnt >= 32 ? 0xFFFFFFFFu : (cnt > 0 ? ((1u << cnt) - 1u) : 0u);
      }
      Z[(int64_t)w * BP + c] = v;
    }
  }
  if (col0 >= d.B) return;
  const uint32_t k0 = (uint32_t)d.seed, k1 = (uint32_t)(d.seed >> 32);
  // pooled tile ch holds items t_lo .. t_lo + cnt - 1 at padded positions 0 .. cnt - 1
  auto tile_items = [&](int ch, int64_t* t_lo, int* cnt) {
    if (ch < d.tx) {
      *t_lo = (int64_t)ch * TILE;
      *cnt = (int)min<int64_t>(TILE, d.nx - *t_lo);
    } else {
      *t_lo = d.nx + (int64_t)(ch - d.tx) * TILE;
      *cnt = (int)min<int64_t>(TILE, n - *t_lo);
    }
  };
  auto draw_tile = [&](int ch, int buf, int first, int stride) {
    int64_t t_lo;
    int cnt;
    tile_items(ch, &t_lo, &cnt);
    // Philox counters t/2 covering the tile's items; a pair may straddle two tiles
    const int64_t c_lo = t_lo >> 1, c_hi = (t_lo + cnt - 1) >> 1;
    const int np = (int)(c_hi - c_lo + 1);
#pragma unroll 2
    for (int q = first; q < np * MSPL; q += stride) {
      const int s = q % MSPL;
      const int64_t ci = c_lo + q / MSPL;
      const uint64_t bb = (uint64_t)(col0 + s);
      if ((int64_t)bb >= d.B) continue;
      const uint4 r = philox4x32_10(make_uint4((uint32_t)ci, (uint32_t)bb,
                                               (uint32_t)(bb >> 32), 0u), k0, k1);
      const int64_t t0 = 2 * ci;
      if (t0 >= t_lo) V[buf][t0 - t_lo][s] = scaled_draw(r.x, r.y, (uint32_t)(n - t0));
      if (t0 + 1 < t_lo + cnt)
        V[buf][t0 + 1 - t_lo][s] = scaled_draw(r.z, r.w, (uint32_t)(n - t0 - 1));
    }
    for (int q = first; q < (TILE - cnt) * MSPL; q += stride)
      V[buf][cnt + q / MSPL][q % MSPL] = 0xFFFFFFFFu;
  };
  draw_tile(0, 0, tid, MTHREADS);
  __syncthreads();
  // Selection scan.  Because v_t <= n - t - 1, the test v_t < need already keeps
  // every remaining item once need == n - t and none once need == 0.
  const int64_t b = col0 + lane;
  const bool drawn = lane < MSPL && b < d.B;
  uint32_t need = (uint32_t)d.nx;
  for (int ch = 0; ch < d.nt; ++ch) {
    if (wave != 0) {
      if (ch + 1 < d.nt) draw_tile(ch + 1, (ch + 1) & 1, tid - 64, MTHREADS - 64);
    } else if (drawn) {
      const uint32_t(*Vb)[MSPL] = V[ch & 1];
#pragma unroll
      for (int w = 0; w < TILE_WORDS; ++w) {
        uint32_t word = 0;
#pragma unroll
        for (int k8 = 0; k8 < 32; k8 += 8) {
          uint32_t v[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] = Vb[32 * w + k8 + e][lane];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t take = v[e] < need ? 1u : 0u;
            need -= take;
            word |= take << (k8 + e);
          }
        }
        Z[(int64_t)(ch * TILE_WORDS + w) * BP + b] = word;
      }
    }
    __syncthreads();
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

// blocks: B_pad / MEMBER_SPLITS workgroups per test
void launch_member(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n,
                   bool wide) {
  if (blocks > 0)
    hipLaunchKernelGGL(wide ? k_member<MEMBER_SPLITS_WIDE> : k_member<MEMBER_SPLITS>,
                       dim3((unsigned)blocks), dim3(MTHREADS), 0, st, d, offs, n);
}
void launch_member_public(int64_t nx, int64_t ny, uint64_t seed, int64_t b0, int64_t count,
                          uint32_t* words, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_member_public, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, nx,
                     ny, seed, b0, count, words);
}

}  // namespace et
