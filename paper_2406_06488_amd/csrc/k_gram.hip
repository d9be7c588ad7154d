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

// 16-byte load through a global-address-space pointer.  Operand prefetches use it: a
// generic (flat) load also counts against the LDS wait counter, so the waits for fragment
// reads from LDS would also wait for the next slice's operands and serialise the prefetch.
__device__ inline uint4 gload16(const void* p) {
  typedef __attribute__((ext_vector_type(4))) unsigned int v4;
  const v4 v = *(const __attribute__((address_space(1))) v4*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}

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
  } else if (d.dense) {  // the whole nt x nt grid, row-major
    c.i = (int)(local / d.nt);
    c.j = (int)(local % d.nt);
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

// Tile epilogue shared by the Gram kernels: one stored tile -> one output (D2 false: the
// staged values are block values) or, with D2 true, the staged values are squared
// distances and are turned into the test's own block values and, with has1, into those of
// the MMD test it feeds (each output's values are formed from the staged copy in place,
// once per entry, so no second set of values is held in registers).  put(half) writes rows
// half*64 .. +63 of the tile into tl (row stride TILE_LDS) and is called between barriers;
// fix(half, first) may then rewrite staged entries, each thread only those of its own
// transform slots (f = tid + 256 k: row f / 128, column f % 128).  All 256 threads of the
// workgroup take part.
template <bool D2, class Put, class Fix>
__device__ __attribute__((always_inline)) inline void finish_tile_with(const TileCtx& c, float* tl, Put put, Fix fix,
                                        const BlockOut o0, const BlockOut o1, const bool has1) {
  __shared__ unsigned int tile_max_bits[2];
  const int tid = threadIdx.x;
  float vmax0 = 0.0f, vmax1 = 0.0f;
  auto stage = [&](int half, bool first) __attribute__((always_inline)) {
    __syncthreads();
    put(half);
    __syncthreads();
    fix(half, first);
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
  __syncthreads();  // a previous tile's maxima have been read
  if (tid < 2) tile_max_bits[tid] = 0u;
  // the partner's output first: the test's own output may overwrite the staged source
  // (the super-tile kernels stage from the test's own block tile)
#pragma nounroll
  for (int half = 0; half < 2; ++half) {
    if (D2 && has1) {
      stage(half, true);
      transform(half, o1.kind, o1.gamma);
      emit_half(o1, half, tl, vmax1);
    }
    stage(half, !(D2 && has1));
    if (D2) transform(half, o0.kind, o0.gamma);
    emit_half(o0, half, tl, vmax0);
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    vmax0 = fmaxf(vmax0, __shfl_xor(vmax0, m, 64));
    if (D2) vmax1 = fmaxf(vmax1, __shfl_xor(vmax1, m, 64));
  }
  // non-negative floats order like their bit patterns
  if ((tid & 63) == 0) {
    atomicMax(&tile_max_bits[0], __float_as_uint(vmax0));
    if (D2 && has1) atomicMax(&tile_max_bits[1], __float_as_uint(vmax1));
  }
  __syncthreads();
  if (tid == 0) {
    o0.tmax[0] = __uint_as_float(tile_max_bits[0]);
    o0.tmax[1] = 0.0f;
    if (D2 && has1) {
      o1.tmax[0] = __uint_as_float(tile_max_bits[1]);
      o1.tmax[1] = 0.0f;
    }
  }
}

// 128-tile workgroups: v[mb][nb][e] is the entry of row wm*64 + mb*32 + 8*(e/4) + 4*h + e%4,
// column wn*64 + nb*32 + lr: the waves with wm == half hold half `half`.
template <bool DUAL>
__device__ inline void finish_tile(const TileCtx& c, float* tl, const f32x16 (&v)[2][2], int wm,
                                   int wn, int h, int lr, const BlockOut o0, const BlockOut o1,
                                   const bool has1) {
  auto put = [&](int half) {
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
  };
  finish_tile_with<DUAL>(c, tl, put, [](int, bool) {}, o0, o1, has1);
}

// Gram entry -> squared distance.  d^2 = |w_a|^2 + |w_b|^2 - 2 g; pairs with
// d^2 < 1e-3 (|w_a|^2 + |w_b|^2), where that difference has cancelled most of its
// digits, are recomputed as a direct FP32 difference of the input rows.
// Near pairs: a Gram-based d^2 below 1e-3 of the norm sum has lost most of its digits to
// cancellation; such pairs (off the diagonal, inside the tile) are recomputed as a direct
// FP32 sum of squared differences of the input rows.
__device__ inline bool needs_refine(const TestDesc& d, const TileCtx& c, int r, int col,
                                    float d2, float nr, float nc) {
  return d.refine && r < c.rows_i && col < c.rows_j && !(c.diag && r == col) &&
         d2 < 1e-3f * (nr + nc);
}
__device__ inline float direct_d2(const TestDesc& d, const TileCtx& c, int r, int col) {
  const float* xa = input_row_f32(d, c.i, r);
  const float* xb = input_row_f32(d, c.j, col);
  float s = 0.0f;
  for (int k = 0; k < d.p; ++k) {
    const float df = xa[k] - xb[k];
    s = fmaf(df, df, s);
  }
  return s;
}
__device__ inline float refine_d2(const TestDesc& d, const TileCtx& c, int r, int col, float d2,
                                  float nr, float nc, int* refined) {
  if (needs_refine(d, c, r, col, d2, nr, nc)) {
    d2 = direct_d2(d, c, r, col);
    ++*refined;
  }
  return d2;
}
__device__ inline float gram_d2(const TestDesc& d, const TileCtx& c, int r, int col, float g,
                                float nr, float nc, int* refined) {
  return refine_d2(d, c, r, col, nr + nc - 2.0f * g, nr, nc, refined);
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
// slice (of both staged planes, hi and lo) is loaded into registers while the current one
// is multiplied; the LDS holds 40 KB, so three workgroups fit per CU.
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
  // K-blocked fp16 pairs: tile t starts at t * TILE * 2 p_pad; chunk q (16 coordinates, hi
  // halves then lo halves) of tile row r at (q * TILE + r) * CHUNK_HALVES
  const uint16_t* Wa = (const uint16_t*)d.W + (int64_t)c.i * TILE * 2 * d.p_pad;
  const uint16_t* Wb = (const uint16_t*)d.W + (int64_t)c.j * TILE * 2 * d.p_pad;
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

  // per half, operand and slice (two chunks) 128 rows x 4 pieces of 8 halves: thread tid
  // owns rows (tid >> 2) + 64 s, coordinates c8 .. c8 + 7 of the slice (chunk c8 / 16), hi
  // ([s][0]) and lo ([s][1])
  const int lrow = tid >> 2, c8 = (tid & 3) * 8;
  const uint16_t* ga = Wa + ((c8 >> 4) * TILE + lrow) * CHUNK_HALVES + (c8 & 15);
  const uint16_t* gb = Wb + ((c8 >> 4) * TILE + lrow) * CHUNK_HALVES + (c8 & 15);
  const int64_t rstep = (int64_t)64 * CHUNK_HALVES;
  uint4 pa[2][2], pb[2][2];
  // slice k0 starts at chunk k0 / 16, i.e. 2 k0 TILE halves on
  auto load = [&](int k0) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        pa[s][pl] = gload16(ga + (int64_t)k0 * 2 * TILE + pl * 16 + s * rstep);
        pb[s][pl] = gload16(gb + (int64_t)k0 * 2 * TILE + pl * 16 + s * rstep);
      }
  };
  load(0);
  for (int k0 = 0; k0 < d.p_pad; k0 += KS16) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int off = (lrow + 64 * s) * LDS_ROW_F16 + c8;
      *(uint4*)(Ah + off) = pa[s][0];
      *(uint4*)(Al + off) = pa[s][1];
      *(uint4*)(Bh + off) = pb[s][0];
      *(uint4*)(Bl + off) = pb[s][1];
    }
    __syncthreads();
    if (k0 + KS16 < d.p_pad) load(k0 + KS16);
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
  // K-blocked operand: tile t starts at t * TILE * p_pad; chunk q (32 coordinates) of tile
  // row r at (q * TILE + r) * CHUNK_HALVES
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

  // 1024 pieces of 8 bf16 per operand and 64-wide slice (two chunks): thread tid owns rows
  // (tid >> 3) + 32 s, piece (tid & 7), which lies in chunk (tid & 7) / 4 of the slice; a
  // wave's load covers 8 rows of both chunks, two contiguous 512-byte runs.  The next slice
  // is loaded into registers while the current one is multiplied.
  const int lrow = tid >> 3, c8 = (tid & 7) * 8;
  const uint16_t* ga = Wa + ((c8 >> 5) * TILE + lrow) * CHUNK_HALVES + (c8 & 31);
  const uint16_t* gb = Wb + ((c8 >> 5) * TILE + lrow) * CHUNK_HALVES + (c8 & 31);
  const int64_t rstep = (int64_t)32 * CHUNK_HALVES;
  uint4 pa0 = gload16(ga), pa1 = gload16(ga + rstep);
  uint4 pa2 = gload16(ga + 2 * rstep), pa3 = gload16(ga + 3 * rstep);
  uint4 pb0 = gload16(gb), pb1 = gload16(gb + rstep);
  uint4 pb2 = gload16(gb + 2 * rstep), pb3 = gload16(gb + 3 * rstep);
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
      // slice k0 + 64 starts at chunk (k0 + 64) / 32, i.e. (k0 + 64) * TILE halves on
      const uint16_t* na = ga + (int64_t)(k0 + 64) * TILE;
      const uint16_t* nb2 = gb + (int64_t)(k0 + 64) * TILE;
      pa0 = gload16(na);
      pa1 = gload16(na + rstep);
      pa2 = gload16(na + 2 * rstep);
      pa3 = gload16(na + 3 * rstep);
      pb0 = gload16(nb2);
      pb1 = gload16(nb2 + rstep);
      pb2 = gload16(nb2 + 2 * rstep);
      pb3 = gload16(nb2 + 3 * rstep);
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

// ------------------------------------------------------- 256 x 256 workgroups (super tiles)
// One workgroup per 2 x 2 block of stored tiles: super tile (I, J) of the grid of
// ceil(nt / 2) super rows and columns (I <= J; for cross tests the rectangle of x-side by
// y-side super tiles).  Wave w = (a, b) = (w >> 1, w & 1) owns pooled tile
// (2I + a, 2J + b) and computes it whole with 4 x 4 accumulators of 32 x 32, so every A or
// B fragment it reads from LDS feeds four MFMAs (two in the 128-tile kernels), and the
// 256 operand rows of each side are fetched once per K slice for all four tiles.  The
// accumulators take a CU's whole register file, so one workgroup runs per CU; its epilogue
// could not overlap any MFMA work.  The kernel therefore ends with the raw Gram tile in the
// stored output tile, and k_gram_finish (one workgroup per stored tile, several per CU)
// forms the block values, sums and maxima.  A wave whose tile is not stored (the lower
// tile of a diagonal super tile, a tile past the edge of the grid) loads its share of the
// operands like the others; its products are discarded.
constexpr int SUPER = 2 * TILE;

// (Cross tests, which store no block tile, are never planned on this kernel; the cross
// branch of super_tile keeps the layout consistent with the 128-tile kernels.)
struct SuperTile {
  // pooled tiles of the super row and column halves (-1: none) and the stored tile index
  // of each of the four tiles (-1: not stored); scalar fields with select accessors, so
  // that indexing by a runtime wave index does not move them to memory
  int ti0, ti1, tj0, tj1;
  int64_t t00, t01, t10, t11;
  __device__ int ti(int a) const { return a ? ti1 : ti0; }
  __device__ int tj(int b) const { return b ? tj1 : tj0; }
  __device__ int64_t tidx(int a, int b) const { return a ? (b ? t11 : t10) : (b ? t01 : t00); }
};

__device__ inline SuperTile super_tile(const TestDesc& d, int64_t local) {
  SuperTile s;
  int I, J;
  if (d.cross) {
    const int sy = (d.ty + 1) / 2;
    I = (int)(local / sy);
    J = (int)(local % sy);
    s.ti0 = 2 * I;
    s.ti1 = 2 * I + 1 < d.tx ? 2 * I + 1 : -1;
    s.tj0 = d.tx + 2 * J;
    s.tj1 = 2 * J + 1 < d.ty ? d.tx + 2 * J + 1 : -1;
    auto at = [&](int i, int j) -> int64_t {
      return i >= 0 && j >= 0 ? (int64_t)i * d.ty + (j - d.tx) : -1;
    };
    s.t00 = at(s.ti0, s.tj0);
    s.t01 = at(s.ti0, s.tj1);
    s.t10 = at(s.ti1, s.tj0);
    s.t11 = at(s.ti1, s.tj1);
  } else {
    tile_coords((int)local, (d.nt + 1) / 2, &I, &J);
    s.ti0 = 2 * I;
    s.ti1 = 2 * I + 1 < d.nt ? 2 * I + 1 : -1;
    s.tj0 = 2 * J;
    s.tj1 = 2 * J + 1 < d.nt ? 2 * J + 1 : -1;
    auto at = [&](int i, int j) -> int64_t {
      return i >= 0 && j >= 0 && i <= j ? tile_index(i, j, d.nt) : -1;
    };
    s.t00 = at(s.ti0, s.tj0);
    s.t01 = at(s.ti0, s.tj1);
    s.t10 = at(s.ti1, s.tj0);
    s.t11 = at(s.ti1, s.tj1);
  }
  return s;
}

__device__ inline TileCtx tile_ctx_at(const TestDesc& d, int i, int j, int64_t t) {
  TileCtx c;
  c.t = (int)t;
  c.i = i;
  c.j = j;
  c.rows_i = tile_rows(d, i);
  c.rows_j = tile_rows(d, j);
  c.diag = i == j;
  return c;
}

// Super-tile kernel.  F16 true: the staged operands are fp16 pairs (hi, lo) of the scaled
// centred values, three v_mfma_f32_32x32x16_f16 per product (hi hi, hi lo, lo hi); F16
// false: BF16 operands, v_mfma_f32_32x32x16_bf16.
//
// One K slice is one 64-byte chunk of every row (BF16: 32 coordinates, two K steps; fp16
// pairs: 16 coordinates, one K step, hi and lo).  In the K-blocked staging the chunks of
// 16 consecutive rows are one contiguous kilobyte, which one wave instruction moves
// straight into LDS (global_load_lds, 16 bytes per lane); each side of a slice is 256 rows
// x 64 bytes in LDS.  Within a row the four 16-byte pieces are stored at slot
// piece ^ ((row / 4) % 4), so that the 16 lanes of an MFMA fragment read (16 rows, one
// piece) hit 16 distinct bank groups; the loading lanes fetch their pieces in that permuted
// order, which keeps each load one contiguous kilobyte.  NBUF buffers of one slice each:
// the loads of slice s + NBUF are issued once slice s has been read, one barrier per slice.
template <bool F16>
__global__ void __launch_bounds__(256) k_gram_super(const TestDesc* __restrict__ descs,
                                                    const int64_t* __restrict__ offs,
                                                    int ntests) {
  constexpr int NSTEP = F16 ? 1 : 2;        // K steps of 16 per slice
  constexpr int NPL = F16 ? 2 : 1;          // operand halves per K step (F16: hi, lo)
  constexpr int SIDEP = 256 * 4;            // 16-byte pieces per side and slice
  constexpr int BUFP = 2 * SIDEP;           // pieces per buffer (both sides)
  constexpr int NBUF = 4;
  constexpr int LOADS = 2 * 16 / 4;         // kilobyte loads per wave and slice
  __shared__ __attribute__((aligned(16))) uint4 lds[NBUF * BUFP];
  const int64_t bid = xcd_grouped(blockIdx.x, gridDim.x);
  const int ti_ = find_test(offs, ntests, bid);
  const TestDesc& d = descs[ti_];
  const SuperTile st = super_tile(d, bid - offs[ti_]);
  // the wave index as a scalar, so that per-wave branches stay scalar branches
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63,
            h = lane >> 5, lr = lane & 31;
  const int wa = w >> 1, wb = w & 1;
  const bool active = __builtin_amdgcn_readfirstlane(st.tidx(wa, wb) >= 0 ? 1 : 0) != 0;
  f32x16 acc[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mb][nb][e] = 0.0f;

  // Global sources.  Load f (of 32 per slice) is side f / 16, rows 16 (f % 16) .. + 15 of
  // that side's 256, which lie in its half (f % 16) / 8.  A half past the edge of the grid
  // reads the first half's rows: those products belong to waves whose tiles are not stored,
  // and are discarded.
  const int64_t nch = d.p_pad / (F16 ? 16 : 32);      // slices (chunks per row)
  const int64_t tstride = nch * TILE * CHUNK_HALVES;  // halves per staged tile
  const uint16_t* W = (const uint16_t*)d.W;
  // pooled tile of each side's halves (scalars; a missing half takes the first half's)
  const int tA0 = st.ti0, tA1 = st.ti1 >= 0 ? st.ti1 : st.ti0;
  const int tB0 = st.tj0, tB1 = st.tj1 >= 0 ? st.tj1 : st.tj0;
  // this lane's 16 bytes of a kilobyte load: row lane / 4 of the 16, stored at slot lane % 4,
  // which holds piece (lane % 4) ^ (row / 4) of that row
  const uint32_t lane_src = (uint32_t)(lane >> 2) * CHUNK_HALVES +
                            (uint32_t)(((lane & 3) ^ ((lane >> 4) & 3)) * 8);
  const uint16_t* srcA0 = W + tA0 * tstride + lane_src;
  const uint16_t* srcA1 = W + tA1 * tstride + lane_src;
  const uint16_t* srcB0 = W + tB0 * tstride + lane_src;
  const uint16_t* srcB1 = W + tB1 * tstride + lane_src;
  // issue the loads of slice SL into buffer BUF (this wave's LOADS kilobytes)
#define GS_ISSUE(SL, BUF)                                                                      \
  do {                                                                                         \
    _Pragma("unroll") for (int q = 0; q < LOADS; ++q) {                                        \
      const int f = w * LOADS + q, side = f >> 4, blk = f & 15;                                \
      const uint16_t* src = side ? ((blk >> 3) ? srcB1 : srcB0) : ((blk >> 3) ? srcA1 : srcA0); \
      __builtin_amdgcn_global_load_lds(                                                        \
          src + ((uint32_t)(SL) * (TILE * CHUNK_HALVES) + (uint32_t)(blk & 7) * (16 * CHUNK_HALVES)), \
          (__attribute__((address_space(3))) void*)(lds + (BUF) * BUFP + f * 64), 16, 0, 0);   \
    }                                                                                          \
  } while (0)
  typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;
  const int nslices = (int)nch;
  // Fragment reads.  Row block rb (32 rows) of a side, K step ks, half pl: lane l reads row
  // rb * 32 + l % 32, piece (F16 ? 2 pl : 2 ks) + l / 32, at slot piece ^ ((l / 4) % 4).
  const int sw = (lane >> 2) & 3;
  const int rd0 = lr * 4 + ((h) ^ sw);           // piece h       (BF16 ks 0; F16 hi)
  const int rd1 = lr * 4 + ((2 + h) ^ sw);       // piece 2 + h   (BF16 ks 1; F16 lo)
#define GS_READ(BUF, KS, FA, FB)                                                              \
  do {                                                                                        \
    _Pragma("unroll") for (int pl = 0; pl < NPL; ++pl)                                        \
      _Pragma("unroll") for (int m = 0; m < 4; ++m) {                                         \
        const int rd_ = (F16 ? pl : (KS)) ? rd1 : rd0;                                        \
        FA[pl * 4 + m] = __builtin_bit_cast(                                                  \
            u32x4, lds[(BUF) * BUFP + (wa * 4 + m) * 128 + rd_]);                             \
        FB[pl * 4 + m] = __builtin_bit_cast(                                                  \
            u32x4, lds[(BUF) * BUFP + SIDEP + (wb * 4 + m) * 128 + rd_]);                     \
      }                                                                                       \
  } while (0)
  // wait until at most LATER slices of this wave's loads are in flight (vmcnt in bits 3:0
  // and 15:14; expcnt and lgkmcnt not waited)
#define GS_WAIT(LATER)                                                                        \
  do {                                                                                        \
    if ((LATER) >= 2)                                                                         \
      __builtin_amdgcn_s_waitcnt(0x0F70 | ((2 * LOADS) & 15) | (((2 * LOADS) >> 4) << 14));   \
    else if ((LATER) == 1)                                                                    \
      __builtin_amdgcn_s_waitcnt(0x0F70 | (LOADS & 15) | ((LOADS >> 4) << 14));               \
    else                                                                                      \
      __builtin_amdgcn_s_waitcnt(0x0F70);                                                     \
  } while (0)
  // A plain barrier: a fenced one would also wait for the loads of the later slices.
#define GS_BARRIER()                  \
  do {                                \
    __builtin_amdgcn_sched_barrier(0); \
    __builtin_amdgcn_s_barrier();      \
    __builtin_amdgcn_sched_barrier(0); \
  } while (0)
  // products of row blocks MB0 .. MB1 - 1 with the current fragments; per accumulator the
  // terms keep the order hi hi, hi lo, lo hi
#define GS_MFMA(MB0, MB1)                                                                   \
  do {                                                                                      \
    _Pragma("unroll") for (int mb = (MB0); mb < (MB1); ++mb)                                \
      _Pragma("unroll") for (int term = 0; term < (F16 ? 3 : 1); ++term)                    \
        _Pragma("unroll") for (int nb = 0; nb < 4; ++nb) {                                  \
          if (F16) {                                                                        \
            const f16x8_t x = __builtin_bit_cast(f16x8_t, ca[(term == 2 ? 4 : 0) + mb]);    \
            const f16x8_t y = __builtin_bit_cast(f16x8_t, cb[(term == 1 ? 4 : 0) + nb]);    \
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, acc[mb][nb], 0, 0, 0); \
          } else {                                                                          \
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(                          \
                __builtin_bit_cast(bf16x8, ca[mb]), __builtin_bit_cast(bf16x8, cb[nb]),     \
                acc[mb][nb], 0, 0, 0);                                                      \
          }                                                                                 \
        }                                                                                   \
  } while (0)
  // prologue: slices 0 .. NBUF - 1 in flight; wait for slice 0
#pragma unroll
  for (int u = 0; u < NBUF; ++u)
    if (u < nslices) GS_ISSUE(u, u);
  {
    const int later = min(NBUF - 1, nslices - 1);
    if (later >= 3)
      __builtin_amdgcn_s_waitcnt(0x0F70 | ((3 * LOADS) & 15) | (((3 * LOADS) >> 4) << 14));
    else
      GS_WAIT(later);
  }
  GS_BARRIER();
  u32x4 ca[4 * NPL], cb[4 * NPL], na[4 * NPL], nb_[4 * NPL];
  // Each K step: half the products; then the fragments of the next K step are read (at the
  // last step of a slice, after the slice boundary: own reads of slice sl complete, since
  // its buffer is refilled after the barrier; slice sl + 1 landed in every wave; slice
  // sl + NBUF issued); then the other half of the products, which run while those reads
  // are in flight.
  GS_READ(0, 0, ca, cb);
  for (int sl = 0; sl < nslices; ++sl) {
#pragma unroll
    for (int ks = 0; ks < NSTEP; ++ks) {
      GS_MFMA(0, 2);
      __builtin_amdgcn_sched_barrier(0);
      if (ks + 1 < NSTEP) {
        GS_READ(sl % NBUF, ks + 1, na, nb_);
      } else if (sl + 1 < nslices) {
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        GS_WAIT(min(NBUF - 2, nslices - 2 - sl));
        GS_BARRIER();
        GS_READ((sl + 1) % NBUF, 0, na, nb_);
        __builtin_amdgcn_sched_barrier(0);
        if (sl + NBUF < nslices) GS_ISSUE(sl + NBUF, sl % NBUF);
      }
      __builtin_amdgcn_sched_barrier(0);
      GS_MFMA(2, 4);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < 4 * NPL; ++k) {
        ca[k] = na[k];
        cb[k] = nb_[k];
      }
    }
  }
#undef GS_MFMA
#undef GS_READ
#undef GS_WAIT
#undef GS_BARRIER
#undef GS_ISSUE
  // ---- the raw Gram tile (times 2^(2 * scale_exp) for fp16 pairs), row-major, into the
  // stored output tile; k_gram_finish turns it into the test's block values
  if (active) {
    float* raw = (float*)d.D + st.tidx(wa, wb) * TILE * TILE;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int r = mb * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
          raw[r * TILE + nb * 32 + lr] = acc[mb][nb][e];
        }
  }
}

// Finish of the super-tile Gram: one workgroup per stored tile turns the raw Gram tile
// into the test's block values (and, DUAL, those of the MMD test it feeds).  Each thread
// forms the squared distances of its 8 float4 of a half tile in registers as it loads them
// (the 128-tile kernels' expression d^2 = |a|^2 + |b|^2 - 2 g after the same exact
// power-of-two unscaling; near pairs, d^2 < 1e-3 (|a|^2 + |b|^2), recomputed as direct
// FP32 differences); each output's block values
// are then staged in LDS and emitted by the shared half-tile epilogue, so the outputs equal
// the 128-tile kernels' bit for bit.  Several workgroups share a CU (35 KB of LDS each),
// so this latency-bound pass overlaps itself.
template <bool DUAL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DUAL ? 3 : 4)))
k_gram_finish(const TestDesc* __restrict__ descs,
                                                     const int64_t* __restrict__ offs,
                                                     int ntests) {
  constexpr int NQ = HALF * TILE / 4 / 256;  // float4 per thread and half
  __shared__ __attribute__((aligned(16))) float tl[HALF * TILE_LDS];
  __shared__ float snorm[2 * TILE];
  __shared__ unsigned int tile_max_bits[2];
  const int64_t bid = xcd_grouped(blockIdx.x, gridDim.x);
  const int ti = find_test(offs, ntests, bid);
  const TestDesc& d = descs[ti];
  const TileCtx c = tile_ctx(d, bid - offs[ti]);
  const int tid = threadIdx.x;
  const float4* raw = (const float4*)((const float*)d.D + (int64_t)c.t * TILE * TILE);
  // entry f = tid + 256 k of a half: row f / 32, columns 4 (f % 32) .. + 3
  float4 cur[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) cur[k] = raw[tid + 256 * k];
  {
    const float* nrm = (const float*)d.nrm;
    snorm[tid] = nrm[(int64_t)(tid < TILE ? c.i : c.j) * TILE + (tid & (TILE - 1))];
  }
  if (tid < 2) tile_max_bits[tid] = 0u;
  const float unscale = d.gop == GOP_F16PAIR ? ldexpf(1.0f, -2 * f16_split_exponent(d)) : 1.0f;
  const bool has1 = DUAL && d.pD != nullptr;
  const BlockOut o0 = own_out(d, c), o1 = DUAL ? partner_out(d, c) : o0;
  float vmax0 = 0.0f, vmax1 = 0.0f;
  int refined = 0;
  __syncthreads();  // norms staged
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (half == 1) {
#pragma unroll
      for (int k = 0; k < NQ; ++k) cur[k] = raw[HALF * TILE / 4 + tid + 256 * k];
    }
    float dv[NQ][4];
    uint32_t near = 0u;  // bit 4 k + u: a near pair
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int f = tid + 256 * k, r = half * HALF + (f >> 5), c4 = 4 * (f & 31);
      const float g[4] = {cur[k].x, cur[k].y, cur[k].z, cur[k].w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float nr = snorm[r], nc = snorm[TILE + c4 + u];
        dv[k][u] = nr + nc - 2.0f * (g[u] * unscale);
        if (needs_refine(d, c, r, c4 + u, dv[k][u], nr, nc)) near |= 1u << (4 * k + u);
      }
    }
#pragma nounroll
    for (int out = has1 ? 1 : 0; out >= 0; --out) {
      const BlockOut o = (DUAL && out) ? o1 : o0;
      const int kind = o.kind;
      const double gamma = o.gamma;
      __syncthreads();  // the previous emit has read tl
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const int f = tid + 256 * k, r = half * HALF + (f >> 5), c4 = 4 * (f & 31);
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = block_value_f32(kind, gamma, c, r, c4 + u, dv[k][u]);
        *(float4*)(tl + (f >> 5) * TILE_LDS + c4) = make_float4(v[0], v[1], v[2], v[3]);
      }
      // near pairs: values of the direct FP32 d^2 replace the staged ones
      uint32_t bits = near;
      while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        const int f = tid + 256 * (b >> 2), r = half * HALF + (f >> 5);
        const int col = 4 * (f & 31) + (b & 3);
        tl[(f >> 5) * TILE_LDS + col] =
            block_value_f32(kind, gamma, c, r, col, direct_d2(d, c, r, col));
        if (out == 0) ++refined;
      }
      __syncthreads();
      float vm = 0.0f;  // one emit call site: the maxima combine afterwards
      emit_half(o, half, tl, vm);
      if (DUAL && out) vmax1 = fmaxf(vmax1, vm);
      else vmax0 = fmaxf(vmax0, vm);
    }
  }
  add_refined(d, refined);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    vmax0 = fmaxf(vmax0, __shfl_xor(vmax0, m, 64));
    if (DUAL) vmax1 = fmaxf(vmax1, __shfl_xor(vmax1, m, 64));
  }
  // non-negative floats order like their bit patterns
  if ((tid & 63) == 0) {
    atomicMax(&tile_max_bits[0], __float_as_uint(vmax0));
    if (has1) atomicMax(&tile_max_bits[1], __float_as_uint(vmax1));
  }
  __syncthreads();
  if (tid == 0) {
    o0.tmax[0] = __uint_as_float(tile_max_bits[0]);
    o0.tmax[1] = 0.0f;
    if (has1) {
      o1.tmax[0] = __uint_as_float(tile_max_bits[1]);
      o1.tmax[1] = 0.0f;
    }
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

void launch_gram(int gop, bool super_tiles, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int n, bool dual) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  if (super_tiles) {  // the raw Gram only; launch_gram_finish forms the block values
    if (gop == GOP_F16PAIR)
      hipLaunchKernelGGL(k_gram_super<true>, g, b, 0, st, d, offs, n);
    else if (gop == GOP_BF16)
      hipLaunchKernelGGL(k_gram_super<false>, g, b, 0, st, d, offs, n);
    return;
  }
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

void launch_gram_finish(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs,
                        int n, bool dual) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  if (dual)
    hipLaunchKernelGGL(k_gram_finish<true>, g, b, 0, st, d, offs, n);
  else
    hipLaunchKernelGGL(k_gram_finish<false>, g, b, 0, st, d, offs, n);
}

}  // namespace et
