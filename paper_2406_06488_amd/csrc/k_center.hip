// Double centring of the stored tiles.
//
// Adding f(a) + f(b) to every pooled pair leaves every resampled ED / MMD
// statistic unchanged: each pooled row of eq. (1)'s weights sums to zero
// (-nx/nx^2 + ny/(nx ny) = 0).  With f(a) = -r_a/n + R/(2 n^2), r_a the pooled
// row sum and R their total, the centred matrix has zero row sums, so for a
// split z (1 = member of x*)
//     ED*(z)  = -(1/nx + 1/ny)^2 * z^T Dc z,
//     MMD*(z) = +(1/nx + 1/ny)^2 * z^T Kc z,
// a single quadratic form over the three stored blocks.  Diagonal tiles are
// halved, so that z^T Dc z = 2 * sum over stored tiles (i <= j) of z_i^T T_ij z_j.
//
// FP32/BF16 forms: the centred value v, scaled by the test's power of two 2^e (so that
// |v| <= 2^14), becomes two planes whose products with split bits are exact:
//  FP32 form: hi = fp16(v), lo = fp16((v - hi) 2^11), multiplied by bits worth 1 and
//    2^-11: hi + lo 2^-11 holds v to about 2^-22 of itself;
//  BF16-refined form: hi = fp16(v), lo = e4m3((v - hi) 2^5) (|lo| <= 2^8 < 448), multiplied
//    by bits worth 1 and 2^-5 on the fp8 MFMA: v to about 2^-15 of itself, 3 bytes per entry.
// The hi (and fp16 lo) plane is laid out in v_mfma_f32_32x32x16_f16 A-fragment order:
// fragment (mb, ks) of a tile is 64 lanes x 8 values, lane = row%32 + 32 * ((col%16)/8),
// for rows 32 mb.. and columns 16 ks.. .  The e4m3 plane follows the 32x32x64 fp8
// A-fragment order: fragment (mb, kb) holds rows 32 mb.. and columns 64 kb.., lane
// row%32 + 32 * ((col%64)/32) holding 32 bytes (columns in order), stored as two 16-byte
// halves: [fragment][half][lane][16 bytes].
// FP64 form: one FP64 row-major tile.
#include "common.h"

namespace et {

__device__ inline double center_value(const TestDesc& d, int i, int j, int r, int col, int rows_i,
                                      int rows_j, double v, double inv_n, double c0) {
  if (r >= rows_i || col >= rows_j) return 0.0;
  const int64_t pa = (int64_t)i * TILE + r, pb = (int64_t)j * TILE + col;
  const double ca = (d.rsum[pa * 2] + d.rsum[pa * 2 + 1]) * inv_n;
  const double cb = (d.rsum[pb * 2] + d.rsum[pb * 2 + 1]) * inv_n;
  double x = ((v - ca) - cb) + c0;
  if (i == j) x *= 0.5;
  return x;
}

// FP64 -> FP32, kept as a separate step: folded into the fp16 conversion that follows it,
// it would become one FP64 -> fp16 rounding, which has no hardware instruction.
__device__ inline float to_f32(double x) {
  float f = (float)x;
  asm volatile("" : "+v"(f));
  return f;
}

__device__ inline uint32_t pack_h2(_Float16 a, _Float16 b) {
  return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
}

// One workgroup per half tile (rows 64 rh .. + 63: fragment row blocks 2 rh and 2 rh + 1),
// so that the grid has twice as many workgroups as stored tiles in flight; on grids
// planned with one workgroup per tile (past 2^22 tiles) a workgroup takes both halves.
__global__ void __launch_bounds__(256) k_center_split(const TestDesc* __restrict__ descs,
                                                      const int64_t* __restrict__ offs,
                                                      int ntests) {
  // centring constants of the tile's 128 rows and 128 columns (0 for padding)
  __shared__ double crow[TILE], ccol[TILE];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  const bool halves = offs[ti + 1] - offs[ti] > d.ntiles;  // two workgroups per tile
  const int t = (int)(halves ? local >> 1 : local);
  const int rh0 = halves ? (int)(local & 1) : 0, rh1 = halves ? rh0 + 1 : 2;
  int i, j;
  tile_coords(t, d.nt, &i, &j);
  const int rows_i = tile_rows(d, i), rows_j = tile_rows(d, j);
  const double n = (double)d.nx + (double)d.ny;
  const double inv_n = 1.0 / n;
  const double c0 = d.obs[4] / (n * n);
  const double scale = d.obs[5];
  const double half = i == j ? 0.5 : 1.0;
  const bool f8lo = d.pfmt == PLANES_F16_E4M3;
  {
    const int r = threadIdx.x & (TILE - 1);
    const int blk = threadIdx.x < TILE ? i : j;
    const int64_t pa = (int64_t)blk * TILE + r;
    const double c = (d.rsum[pa * 2] + d.rsum[pa * 2 + 1]) * inv_n;
    if (threadIdx.x < TILE) crow[r] = c;
    else ccol[r] = c;
  }
  __syncthreads();
  const float* Dt = (const float*)d.D + (int64_t)t * TILE * TILE;
  uint8_t* P = (uint8_t*)d.planes + (int64_t)t * plane_bytes_per_entry(d.pfmt) * TILE * TILE;
  uint16_t* Phi = (uint16_t*)P;
  uint8_t* Plo = P + 2 * TILE * TILE;
  for (int rh = rh0; rh < rh1; ++rh) {
    // every load of the thread first (8 x 16 B in flight), then the conversions; fragment
    // q of the half: 8 values of row block q / 512 (2 rh or 2 rh + 1)
    constexpr int NQ = TILE * TILE / 8 / 256 / 2;
    float4 raw[NQ][2];
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int q = rh * (NQ * 256) + threadIdx.x + 256 * it;
      const int mb = q >> 9, ks = (q >> 6) & 7, lane = q & 63;
      const int r = mb * 32 + (lane & 31), c0l = ks * 16 + 8 * (lane >> 5);
      raw[it][0] = *(const float4*)(Dt + r * TILE + c0l);
      raw[it][1] = *(const float4*)(Dt + r * TILE + c0l + 4);
    }
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int q = rh * (NQ * 256) + threadIdx.x + 256 * it;
      const int mb = q >> 9, ks = (q >> 6) & 7, lane = q & 63;
      const int r = mb * 32 + (lane & 31), c0l = ks * 16 + 8 * (lane >> 5);
      const float v[8] = {raw[it][0].x, raw[it][0].y, raw[it][0].z, raw[it][0].w,
                          raw[it][1].x, raw[it][1].y, raw[it][1].z, raw[it][1].w};
      const double ca = crow[r];
      _Float16 hi[8], lo[8];
      uint32_t lo8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int col = c0l + e;
        double x = 0.0;
        if (r < rows_i && col < rows_j) x = ((((double)v[e] - ca) - ccol[col]) + c0) * half * scale;
        // FP64 -> FP32 -> fp16 (both hardware conversions; a direct FP64 -> fp16 rounding is
        // a long software sequence): hi may then round one way twice, which the low plane
        // absorbs, since it is formed from the exact FP64 remainder x - hi
        hi[e] = (_Float16)to_f32(x);
        const double rem = x - (double)(float)hi[e];
        if (f8lo) lo8[e] = f32_to_e4m3(to_f32(rem * 32.0));
        else lo[e] = (_Float16)to_f32(rem * 2048.0);
      }
      uint4 w;
      w.x = pack_h2(hi[0], hi[1]); w.y = pack_h2(hi[2], hi[3]);
      w.z = pack_h2(hi[4], hi[5]); w.w = pack_h2(hi[6], hi[7]);
      *(uint4*)(Phi + (int64_t)q * 8) = w;
      if (f8lo) {
        // columns c0l .. c0l+7 are bytes (c0l % 16) .. +7 of half (c0l % 32) / 16 of lane
        // (r % 32) + 32 ((c0l % 64) / 32) in fragment (mb, c0l / 64)
        const int kb = c0l >> 6, g = (c0l >> 5) & 1, hf = (c0l >> 4) & 1;
        const int64_t off = ((int64_t)((mb * 2 + kb) * 2 + hf) * 64 + (lane & 31) + 32 * g) * 16 +
                            (c0l & 15);
        uint2 b;
        b.x = lo8[0] | (lo8[1] << 8) | (lo8[2] << 16) | (lo8[3] << 24);
        b.y = lo8[4] | (lo8[5] << 8) | (lo8[6] << 16) | (lo8[7] << 24);
        *(uint2*)(Plo + off) = b;
      } else {
        w.x = pack_h2(lo[0], lo[1]); w.y = pack_h2(lo[2], lo[3]);
        w.z = pack_h2(lo[4], lo[5]); w.w = pack_h2(lo[6], lo[7]);
        *(uint4*)(Phi + TILE * TILE + (int64_t)q * 8) = w;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_center_f64(const TestDesc* __restrict__ descs,
                                                    const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int t = (int)(blockIdx.x - offs[ti]);
  int i, j;
  tile_coords(t, d.nt, &i, &j);
  const int rows_i = tile_rows(d, i), rows_j = tile_rows(d, j);
  const double n = (double)d.nx + (double)d.ny;
  const double inv_n = 1.0 / n;
  const double c0 = d.obs[4] / (n * n);
  const double* Dt = (const double*)d.D + (int64_t)t * TILE * TILE;
  double* P = (double*)d.planes + (int64_t)t * TILE * TILE;
  for (int e = threadIdx.x; e < TILE * TILE; e += 256) {
    const int r = e / TILE, col = e % TILE;
    P[e] = center_value(d, i, j, r, col, rows_i, rows_j, Dt[e], inv_n, c0);
  }
}

void launch_center(bool f64, int64_t blocks, hipStream_t st, const TestDesc* d,
                   const int64_t* offs, int n) {
  if (blocks <= 0) return;
  if (f64) hipLaunchKernelGGL(k_center_f64, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
  else hipLaunchKernelGGL(k_center_split, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}

}  // namespace et
