// Block stage: every stored tile (i <= j) of the pooled tile grid is one
// workgroup.  FP32 / BF16 forms: Gram tile G = W_i W_j^T on MFMA, epilogue
// d^2 = |w_a|^2 + |w_b|^2 - 2 g (clamped at 0), then D = sqrt(d^2) (energy
// distance, Alg. 3) or K = exp(-gamma d^2) (Gaussian kernel).  The BF16 form
// recomputes pairs with d^2 < 1e-3 (|w_a|^2 + |w_b|^2) as a direct FP32
// difference of the input rows.  The FP64 form evaluates Alg. 3 as written
// (sum of squared differences) on the vector ALU.
//
// Every stored tile also yields FP64 row sums and column sums, from which the
// observed statistic (eq. 1 / eq. 2) and the double-centring constants follow.
#include "common.h"

namespace et {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LDS_ROW_BF16 = 72;  // 64 staged k + 8 pad (bf16)

struct TileCtx {
  int t, i, j;
  int rows_i, rows_j;
  bool diag;
};

__device__ inline TileCtx tile_ctx(const TestDesc& d, int64_t local) {
  TileCtx c;
  c.t = (int)local;
  if (d.cross) {  // the rectangle x side by y side, row-major
    c.i = (int)(local / d.ty);
    c.j = d.tx + (int)(local % d.ty);
  } else {
    tile_coords(c.t, d.nt, &c.i, &c.j);
  }
  c.rows_i = tile_rows(d, c.i);
  c.rows_j = tile_rows(d, c.j);
  c.diag = c.i == c.j;
  return c;
}

// Input row (pooled, unpadded) of tile row r of pooled tile i.
__device__ inline const float* input_row_f32(const TestDesc& d, int i, int r) {
  const int64_t t = i < d.tx ? (int64_t)i * TILE + r : d.nx + (int64_t)(i - d.tx) * TILE + r;
  return pooled_row<float>(d, t);
}

// d^2 -> stored block value (distance, or Gaussian kernel with bandwidth 1 / gamma);
// padding rows/columns hold 0.
__device__ inline float block_value_f32(int kind, double gamma, const TileCtx& c, int r, int col,
                                        float d2) {
  if (r >= c.rows_i || col >= c.rows_j) return 0.0f;
  if (c.diag && r == col) return kind == KIND_ED ? 0.0f : 1.0f;
  d2 = fmaxf(d2, 0.0f);
  return kind == KIND_ED ? sqrtf(d2) : expf((float)(-gamma) * d2);
}

// The block outputs one epilogue pass writes: the test's own, or those of the MMD test it
// feeds (shared block stage).
struct BlockOut {
  int kind;
  int split;  // cross tests: y-side columns below `split` are x2, the rest y2; -1 otherwise
  double gamma;
  float* D;
  double* tsum;
  float* tmax;
};
// columns of y-side tile j that hold x2 rows (cross tests)
__device__ inline int cross_split(const TestDesc& d, int j) {
  const int s = d.cnx2 - (j - d.tx) * TILE;
  return s < 0 ? 0 : (s > TILE ? TILE : s);
}
__device__ inline BlockOut own_out(const TestDesc& d, const TileCtx& c) {
  const int64_t t = c.t;
  return BlockOut{d.kind, d.cross ? cross_split(d, c.j) : -1, d.gamma,
                  d.cross ? nullptr : (float*)d.D + t * TILE * TILE,
                  d.tsum + t * TSUM_STRIDE, d.tmax + t * TMAX_PER_TILE};
}
__device__ inline BlockOut partner_out(const TestDesc& d, const TileCtx& c) {
  const int64_t t = c.t;
  return BlockOut{KIND_MMD, -1, d.pgamma, (float*)d.pD + t * TILE * TILE,
                  d.ptsum + t * TSUM_STRIDE, d.ptmax + t * TMAX_PER_TILE};
}

constexpr int HALF = TILE / 2;

// Epilogue through LDS, half a tile (64 rows) at a time, so a workgroup needs ~34 KB of LDS
// for it.  Row stride 132 floats: rows stay 16-byte aligned for vector reads, and the bank
// of (row, col) is (4 row + col) % 32, which the patterns below keep distinct within every
// 32 lanes.
constexpr int TILE_LDS = TILE + 4;

// Staged half tile (64 rows of block values) -> FP64 row sums, FP64 column sums of the
// half, the stored rows and the running max |value|.  All 256 threads take part:
//  row sums: four threads per row, thread q reading columns q*32 + (k + q) % 32;
//  column sums: two threads per column in one wave (rows 0..31 and 32..63);
//  store: float4 reads of whole rows (32 lanes per row), coalesced float4 stores.
__device__ inline void emit_half(const BlockOut& o, int half, const float* tl, float& vmax) {
  const int tid = threadIdx.x;
  if (o.split >= 0) {
    // cross tests: each row's sums over the x2 columns and over the y2 columns, kept apart
    // (tsum[r] and tsum[TILE + r]); the tile itself is not stored
    const int row = tid >> 2, q = tid & 3;
    const float* src = tl + row * TILE_LDS + q * 32;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const int col = q * 32 + ((k + q) & 31);
      const float x = src[(k + q) & 31];
      if (col < o.split) s0 += (double)x;
      else s1 += (double)x;
      vmax = fmaxf(vmax, fabsf(x));
    }
    s0 += __shfl_xor(s0, 1, 64);
    s0 += __shfl_xor(s0, 2, 64);
    s1 += __shfl_xor(s1, 1, 64);
    s1 += __shfl_xor(s1, 2, 64);
    if (q == 0) {
      o.tsum[half * HALF + row] = s0;
      o.tsum[TILE + half * HALF + row] = s1;
    }
    return;
  }
  {
    const int row = tid >> 2, q = tid & 3;
    const float* src = tl + row * TILE_LDS + q * 32;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const float x = src[(k + q) & 31];
      s += (double)x;
      vmax = fmaxf(vmax, fabsf(x));
    }
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (q == 0) o.tsum[half * HALF + row] = s;
  }
  {
    const int col = (tid >> 6) * 32 + (tid & 31), part = (tid >> 5) & 1;
    const float* src = tl + part * 32 * TILE_LDS + col;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < 32; ++k) s += (double)src[k * TILE_LDS];
    s += __shfl_xor(s, 32, 64);
    if (part == 0) o.tsum[TILE * (1 + half) + col] = s;
  }
  float4* dst = (float4*)(o.D + half * HALF * TILE);
#pragma unroll
  for (int k = 0; k < HALF * TILE / 4 / 256; ++k) {
    const int f = tid + 256 * k;
    dst[f] = *(const float4*)(tl + (f >> 5) * TILE_LDS + 4 * (f & 31));
  }
}

// Full tile in registers -> one output (DUAL false: v holds its block values) or the
// test's own output and, with has1, the MMD test it feeds (DUAL true: v holds squared
// distances; each output's values are formed from the staged copy in place, once per
// entry, so no second set of values is held in registers).  v[mb][nb][e] is the entry of
// row wm*64 + mb*32 + 8*(e/4) + 4*h + e%4, column wn*64 + nb*32 + lr: the waves with
// wm == half hold half `half`.
template <bool DUAL>
__device__ inline void finish_tile(const TileCtx& c, float* tl, const f32x16 (&v)[2][2], int wm,
                                   int wn, int h, int lr, const BlockOut o0, const BlockOut o1,
                                   const bool has1) {
  __shared__ unsigned int tile_max_bits[2];
  const int tid = threadIdx.x;
  float vmax0 = 0.0f, vmax1 = 0.0f;
  auto stage = [&](int half) {
    __syncthreads();
    if (wm == half) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int r = mb * 32 + 8 * (e >> 2) + 4 * h + (e & 3);  // row within the half
            tl[r * TILE_LDS + wn * 64 + nb * 32 + lr] = v[mb][nb][e];
          }
    }
    __syncthreads();
  };
  auto transform = [&](int half, int kind, double gamma) {
#pragma unroll 2
    for (int k = 0; k < HALF * TILE / 256; ++k) {
      const int f = tid + 256 * k, r = f >> 7, col = f & (TILE - 1);
      float* q = tl + r * TILE_LDS + col;
      *q = block_value_f32(kind, gamma, c, half * HALF + r, col, *q);
    }
    __syncthreads();
  };
  if (tid < 2) tile_max_bits[tid] = 0u;
#pragma nounroll
  for (int half = 0; half < 2; ++half) {
    stage(half);
    if (DUAL) transform(half, o0.kind, o0.gamma);
    emit_half(o0, half, tl, vmax0);
    if (DUAL && has1) {
      stage(half);
      transform(half, o1.kind, o1.gamma);
      emit_half(o1, half, tl, vmax1);
    }
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    vmax0 = fmaxf(vmax0, __shfl_xor(vmax0, m, 64));
    if (DUAL) vmax1 = fmaxf(vmax1, __shfl_xor(vmax1, m, 64));
  }
  // non-negative floats order like their bit patterns
  if ((tid & 63) == 0) {
    atomicMax(&tile_max_bits[0], __float_as_uint(vmax0));
    if (DUAL && has1) atomicMax(&tile_max_bits[1], __float_as_uint(vmax1));
  }
  __syncthreads();
  if (tid == 0) {
    o0.tmax[0] = __uint_as_float(tile_max_bits[0]);
    o0.tmax[1] = 0.0f;
    if (DUAL && has1) {
      o1.tmax[0] = __uint_as_float(tile_max_bits[1]);
      o1.tmax[1] = 0.0f;
    }
  }
}

// Gram entry -> squared distance.  d^2 = |w_a|^2 + |w_b|^2 - 2 g; pairs with
// d^2 < 1e-3 (|w_a|^2 + |w_b|^2), where that difference has cancelled most of its
// digits, are recomputed as a direct FP32 difference of the input rows.
__device__ inline float gram_d2(const TestDesc& d, const TileCtx& c, int r, int col, float g,
                                float nr, float nc, int* refined) {
  float d2 = nr + nc - 2.0f * g;
  if (d.refine && r < c.rows_i && col < c.rows_j && !(c.diag && r == col) &&
      d2 < 1e-3f * (nr + nc)) {
    const float* xa = input_row_f32(d, c.i, r);
    const float* xb = input_row_f32(d, c.j, col);
    float s = 0.0f;
    for (int k = 0; k < d.p; ++k) {
      const float df = xa[k] - xb[k];
      s = fmaf(df, df, s);
    }
    d2 = s;
    ++*refined;
  }
  return d2;
}

__device__ inline void add_refined(const TestDesc& d, int refined) {
  if (!refined) return;
  atomicAdd(&d.flags[1], refined);
  if (d.pflags) atomicAdd(&d.pflags[1], refined);
}

// Gram entries of a full-tile workgroup (2 x 2 waves of 64 x 64) -> squared distances
// (VALUES false) or the test's own block values (VALUES true), in place.
template <bool VALUES>
__device__ inline void gram_epilogue(const TestDesc& d, const TileCtx& c, f32x16 (&acc)[2][2],
                                     int wm, int wn, int h, int lr) {
  // the tile's 128 row norms and 128 column norms, staged once instead of two global
  // loads per entry
  __shared__ float snorm[2 * TILE];
  const int tid = threadIdx.x;
  {
    const float* nrm = (const float*)d.nrm;
    snorm[tid] = nrm[(int64_t)(tid < TILE ? c.i : c.j) * TILE + (tid & (TILE - 1))];
  }
  __syncthreads();
  int refined = 0;
  for (int mb = 0; mb < 2; ++mb)
    for (int nb = 0; nb < 2; ++nb) {
      const int col = wn * 64 + nb * 32 + lr;
      const float nc = snorm[TILE + col];
      for (int e = 0; e < 16; ++e) {
        const int r = wm * 64 + mb * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
        const float d2 = gram_d2(d, c, r, col, acc[mb][nb][e], snorm[r], nc, &refined);
        acc[mb][nb][e] = VALUES ? block_value_f32(d.kind, d.gamma, c, r, col, d2) : d2;
      }
    }
  add_refined(d, refined);
}

// ------------------------------------------- fp16-pair operands (FP32-accurate) on fp16 MFMA
// The staged operand holds fp16 pairs (hi, lo) of w 2^e (22 significant bits; see
// f16_split_exponent).  Each Gram entry is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b
// (the lo_a lo_b term, 2^-22 of the product, is dropped) with three
// v_mfma_f32_32x32x16_f16 into one FP32 accumulator: all three products are exact in FP32,
// so the entry carries the same FP32 accumulation rounding as an FP32 Gram, at the fp16
// MFMA rate.  The accumulator is scaled back by 2^-2e before the epilogue.
// 4 waves as 2 x 2, each 64 x 64 = 2 x 2 blocks of 32 x 32; K slices of 32 pairs; the next
// slice is loaded into registers while the current one is multiplied; the pairs are split
// into a hi and a lo plane when stored to LDS (40 KB), so three workgroups fit per CU.
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
constexpr int KS16 = 32;                // pairs per K slice
constexpr int LDS_ROW_F16 = KS16 + 8;   // halves per LDS row (80 bytes)

template <bool DUAL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_gram_f16x3(const TestDesc* __restrict__ descs, const int64_t* __restrict__ offs, int ntests) {
  __shared__ __attribute__((aligned(16))) float smem[HALF * TILE_LDS > 2 * TILE * LDS_ROW_F16
                                                         ? HALF * TILE_LDS
                                                         : 2 * TILE * LDS_ROW_F16];
  const int64_t bid = xcd_grouped(blockIdx.x, gridDim.x);
  const int ti = find_test(offs, ntests, bid);
  const TestDesc d = descs[ti];
  const TileCtx c = tile_ctx(d, bid - offs[ti]);
  const uint32_t* Wa = (const uint32_t*)d.W + (int64_t)c.i * TILE * d.p_pad;
  const uint32_t* Wb = (const uint32_t*)d.W + (int64_t)c.j * TILE * d.p_pad;
  uint16_t* Ah = (uint16_t*)smem;
  uint16_t* Al = Ah + TILE * LDS_ROW_F16;
  uint16_t* Bh = Al + TILE * LDS_ROW_F16;
  uint16_t* Bl = Bh + TILE * LDS_ROW_F16;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wm = w >> 1, wn = w & 1, h = lane >> 5, lr = lane & 31;
  f32x16 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  // 1024 uint4 (4 pairs each) per operand and slice: thread tid owns rows (tid >> 3) + 32 s,
  // pairs 4 (tid & 7) .. +3
  const int lrow = tid >> 3, c4 = (tid & 7) * 4;
  const uint32_t* ga = Wa + (int64_t)lrow * d.p_pad + c4;
  const uint32_t* gb = Wb + (int64_t)lrow * d.p_pad + c4;
  const int64_t rstep = (int64_t)32 * d.p_pad;
  uint4 pa[4], pb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    pa[s] = *(const uint4*)(ga + s * rstep);
    pb[s] = *(const uint4*)(gb + s * rstep);
  }
  // four pairs -> their four hi halves and four lo halves
  auto split_store = [&](const uint4 q, uint16_t* hi, uint16_t* lo) {
    uint2 vh, vl;
    vh.x = (q.x & 0xFFFFu) | (q.y << 16);
    vh.y = (q.z & 0xFFFFu) | (q.w << 16);
    vl.x = (q.x >> 16) | (q.y & 0xFFFF0000u);
    vl.y = (q.z >> 16) | (q.w & 0xFFFF0000u);
    *(uint2*)hi = vh;
    *(uint2*)lo = vl;
  };
  for (int k0 = 0; k0 < d.p_pad; k0 += KS16) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int off = (lrow + 32 * s) * LDS_ROW_F16 + c4;
      split_store(pa[s], Ah + off, Al + off);
      split_store(pb[s], Bh + off, Bl + off);
    }
    __syncthreads();
    if (k0 + KS16 < d.p_pad) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        pa[s] = *(const uint4*)(ga + k0 + KS16 + s * rstep);
        pb[s] = *(const uint4*)(gb + k0 + KS16 + s * rstep);
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS16 / 16; ++ks) {
      f16x8_t ah[2], al[2], bh[2], bl[2];
      for (int mb = 0; mb < 2; ++mb) {
        const int off = (wm * 64 + mb * 32 + lr) * LDS_ROW_F16 + 16 * ks + 8 * h;
        ah[mb] = *(const f16x8_t*)(Ah + off);
        al[mb] = *(const f16x8_t*)(Al + off);
      }
      for (int nb = 0; nb < 2; ++nb) {
        const int off = (wn * 64 + nb * 32 + lr) * LDS_ROW_F16 + 16 * ks + 8 * h;
        bh[nb] = *(const f16x8_t*)(Bh + off);
        bl[nb] = *(const f16x8_t*)(Bl + off);
      }
      for (int mb = 0; mb < 2; ++mb)
        for (int nb = 0; nb < 2; ++nb) {
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mb], bh[nb], acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mb], bl[nb], acc[mb][nb], 0, 0, 0);
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[mb], bh[nb], acc[mb][nb], 0, 0, 0);
        }
    }
  }
  const float unscale = ldexpf(1.0f, -2 * f16_split_exponent(d));
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 16; ++e) acc[a][b][e] *= unscale;
  // DUAL: launches that hold a test feeding an MMD test keep the squared distances for two
  // outputs; plain launches turn them into block values at once
  if (DUAL) {
    gram_epilogue<false>(d, c, acc, wm, wn, h, lr);
    finish_tile<true>(c, smem, acc, wm, wn, h, lr, own_out(d, c), partner_out(d, c),
                      d.pD != nullptr);
  } else {
    gram_epilogue<true>(d, c, acc, wm, wn, h, lr);
    const BlockOut o = own_out(d, c);
    finish_tile<false>(c, smem, acc, wm, wn, h, lr, o, o, false);
  }
}

// ---------------------------------------------------------------- BF16 MFMA
// Same arrangement with v_mfma_f32_32x32x16_bf16; pairs whose Gram-based d^2
// falls below 1e-3 of the norm sum are recomputed from the FP32 input rows.
template <bool DUAL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_gram_bf16(const TestDesc* __restrict__ descs,
                                                   const int64_t* __restrict__ offs, int ntests) {
  __shared__ __attribute__((aligned(16))) float smem[HALF * TILE_LDS > TILE * LDS_ROW_BF16 ? HALF * TILE_LDS
                                                              : TILE * LDS_ROW_BF16];
  const int64_t bid = xcd_grouped(blockIdx.x, gridDim.x);
  const int ti = find_test(offs, ntests, bid);
  const TestDesc d = descs[ti];
  const TileCtx c = tile_ctx(d, bid - offs[ti]);
  const uint16_t* Wa = (const uint16_t*)d.W + (int64_t)c.i * TILE * d.p_pad;
  const uint16_t* Wb = (const uint16_t*)d.W + (int64_t)c.j * TILE * d.p_pad;
  uint16_t* As = (uint16_t*)smem;
  uint16_t* Bs = As + TILE * LDS_ROW_BF16;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wm = w >> 1, wn = w & 1, h = lane >> 5, lr = lane & 31;
  f32x16 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.0f;

  // 1024 chunks of 8 bf16 per operand and 64-wide slice: thread tid owns rows
  // (tid >> 3) + 32 s, chunk (tid & 7); the next slice is loaded into registers while the
  // current one is multiplied.
  const int lrow = tid >> 3, c8 = (tid & 7) * 8;
  const uint16_t* ga = Wa + (int64_t)lrow * d.p_pad + c8;
  const uint16_t* gb = Wb + (int64_t)lrow * d.p_pad + c8;
  const int64_t rstep = (int64_t)32 * d.p_pad;
  uint4 pa0 = *(const uint4*)(ga), pa1 = *(const uint4*)(ga + rstep);
  uint4 pa2 = *(const uint4*)(ga + 2 * rstep), pa3 = *(const uint4*)(ga + 3 * rstep);
  uint4 pb0 = *(const uint4*)(gb), pb1 = *(const uint4*)(gb + rstep);
  uint4 pb2 = *(const uint4*)(gb + 2 * rstep), pb3 = *(const uint4*)(gb + 3 * rstep);
  for (int k0 = 0; k0 < d.p_pad; k0 += 64) {
    __syncthreads();
    uint16_t* la = As + lrow * LDS_ROW_BF16 + c8;
    uint16_t* lb = Bs + lrow * LDS_ROW_BF16 + c8;
    *(uint4*)(la) = pa0;
    *(uint4*)(la + 32 * LDS_ROW_BF16) = pa1;
    *(uint4*)(la + 64 * LDS_ROW_BF16) = pa2;
    *(uint4*)(la + 96 * LDS_ROW_BF16) = pa3;
    *(uint4*)(lb) = pb0;
    *(uint4*)(lb + 32 * LDS_ROW_BF16) = pb1;
    *(uint4*)(lb + 64 * LDS_ROW_BF16) = pb2;
    *(uint4*)(lb + 96 * LDS_ROW_BF16) = pb3;
    __syncthreads();
    if (k0 + 64 < d.p_pad) {
      const uint16_t* na = ga + k0 + 64;
      const uint16_t* nb2 = gb + k0 + 64;
      pa0 = *(const uint4*)(na);
      pa1 = *(const uint4*)(na + rstep);
      pa2 = *(const uint4*)(na + 2 * rstep);
      pa3 = *(const uint4*)(na + 3 * rstep);
      pb0 = *(const uint4*)(nb2);
      pb1 = *(const uint4*)(nb2 + rstep);
      pb2 = *(const uint4*)(nb2 + 2 * rstep);
      pb3 = *(const uint4*)(nb2 + 3 * rstep);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8 av[2], bv[2];
      for (int mb = 0; mb < 2; ++mb)
        av[mb] = *(const bf16x8*)(As + (wm * 64 + mb * 32 + lr) * LDS_ROW_BF16 + 16 * s + 8 * h);
      for (int nb = 0; nb < 2; ++nb)
        bv[nb] = *(const bf16x8*)(Bs + (wn * 64 + nb * 32 + lr) * LDS_ROW_BF16 + 16 * s + 8 * h);
      for (int mb = 0; mb < 2; ++mb)
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] =
              __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
    }
  }
  // DUAL: launches that hold a test feeding an MMD test keep the squared distances for two
  // outputs; plain launches turn them into block values at once
  if (DUAL) {
    gram_epilogue<false>(d, c, acc, wm, wn, h, lr);
    finish_tile<true>(c, smem, acc, wm, wn, h, lr, own_out(d, c), partner_out(d, c),
                      d.pD != nullptr);
  } else {
    gram_epilogue<true>(d, c, acc, wm, wn, h, lr);
    const BlockOut o = own_out(d, c);
    finish_tile<false>(c, smem, acc, wm, wn, h, lr, o, o, false);
  }
}

// ---------------------------------------------------------------- FP64 direct
// Alg. 3 literally: sum over k of (x_ak - y_bk)^2 on the FP64 vector ALU.
// Thread (tr, tc) owns rows tr + 16 a and columns tc + 16 b (a, b < 8).
constexpr int KC64 = 16;
__global__ void __launch_bounds__(256) k_dist_f64(const TestDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ offs, int ntests) {
  __shared__ double As[TILE * (KC64 + 1)];
  __shared__ double Bs[TILE * (KC64 + 1)];
  __shared__ double rp[TILE * 16];
  __shared__ double cp[16 * TILE];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const TileCtx c = tile_ctx(d, blockIdx.x - offs[ti]);
  const double* Wa = (const double*)d.W + (int64_t)c.i * TILE * d.p_pad;
  const double* Wb = (const double*)d.W + (int64_t)c.j * TILE * d.p_pad;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double acc[8][8];
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
  for (int k0 = 0; k0 < d.p_pad; k0 += KC64) {
    __syncthreads();
    for (int e = tid; e < TILE * KC64; e += 256) {
      const int row = e / KC64, k = e % KC64;
      As[row * (KC64 + 1) + k] = Wa[(int64_t)row * d.p_pad + k0 + k];
      Bs[row * (KC64 + 1) + k] = Wb[(int64_t)row * d.p_pad + k0 + k];
    }
    __syncthreads();
    for (int k = 0; k < KC64; ++k) {
      double av[8], bv[8];
      for (int a = 0; a < 8; ++a) av[a] = As[(tr + 16 * a) * (KC64 + 1) + k];
      for (int b = 0; b < 8; ++b) bv[b] = Bs[(tc + 16 * b) * (KC64 + 1) + k];
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
          const double df = av[a] - bv[b];
          acc[a][b] = fma(df, df, acc[a][b]);
        }
    }
  }
  // cross tests: row sums over the x2 columns (rs) and the y2 columns (cs, in place of the
  // column sums), no stored tile
  const int split = d.cross ? cross_split(d, c.j) : -1;
  double* D = d.cross ? nullptr : (double*)d.D + (int64_t)c.t * TILE * TILE;
  double rs[8], cs[8];
  for (int a = 0; a < 8; ++a) rs[a] = 0.0;
  for (int b = 0; b < 8; ++b) cs[b] = 0.0;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      const int r = tr + 16 * a, col = tc + 16 * b;
      double v;
      if (r >= c.rows_i || col >= c.rows_j) v = 0.0;
      else if (c.diag && r == col) v = d.kind == KIND_ED ? 0.0 : 1.0;
      else v = d.kind == KIND_ED ? sqrt(acc[a][b]) : exp(-d.gamma * acc[a][b]);
      if (split >= 0) {
        if (col < split) rs[a] += v;
        else cs[a] += v;
      } else {
        D[r * TILE + col] = v;
        rs[a] += v;
        cs[b] += v;
      }
    }
  if (split >= 0) {
    for (int a = 0; a < 8; ++a) rp[(tr + 16 * a) * 16 + tc] = rs[a];
    for (int a = 0; a < 8; ++a) cp[(tr + 16 * a) * 16 + tc] = cs[a];
    __syncthreads();
    if (tid < TILE) {
      double s0 = 0.0, s1 = 0.0;
      for (int q = 0; q < 16; ++q) {
        s0 += rp[tid * 16 + q];
        s1 += cp[tid * 16 + q];
      }
      d.tsum[(int64_t)c.t * TSUM_STRIDE + tid] = s0;
      d.tsum[(int64_t)c.t * TSUM_STRIDE + TILE + tid] = s1;
    }
    return;
  }
  for (int a = 0; a < 8; ++a) rp[(tr + 16 * a) * 16 + tc] = rs[a];
  for (int b = 0; b < 8; ++b) cp[tr * TILE + tc + 16 * b] = cs[b];
  __syncthreads();
  double s = 0.0;
  if (tid < TILE) {
    for (int q = 0; q < 16; ++q) s += rp[tid * 16 + q];
    d.tsum[(int64_t)c.t * TSUM_STRIDE + tid] = s;
  } else {
    const int col = tid - TILE;
    for (int q = 0; q < 16; ++q) s += cp[q * TILE + col];
    d.tsum[(int64_t)c.t * TSUM_STRIDE + TILE + col] = s;  // all 128 rows in one slot
    d.tsum[(int64_t)c.t * TSUM_STRIDE + 2 * TILE + col] = 0.0;
  }
}

void launch_gram(int gop, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int n, bool dual) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  if (gop == GOP_F64)
    hipLaunchKernelGGL(k_dist_f64, g, b, 0, st, d, offs, n);
  else if (gop == GOP_F16PAIR && dual)
    hipLaunchKernelGGL(k_gram_f16x3<true>, g, b, 0, st, d, offs, n);
  else if (gop == GOP_F16PAIR)
    hipLaunchKernelGGL(k_gram_f16x3<false>, g, b, 0, st, d, offs, n);
  else if (dual)
    hipLaunchKernelGGL(k_gram_bf16<true>, g, b, 0, st, d, offs, n);
  else
    hipLaunchKernelGGL(k_gram_bf16<false>, g, b, 0, st, d, offs, n);
}

}  // namespace et
