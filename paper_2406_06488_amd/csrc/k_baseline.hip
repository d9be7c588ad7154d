// The two baselines the efficient test is measured against, on the same chip:
//  - the standard permutation test (Alg. 4): every split's statistic recomputed from
//    distance (or kernel) blocks of its own X*, Y*;
//  - the pre-computation test (Alg. 5): the distance (kernel) matrix of the pooled sample
//    once, then per split the sums of the entries its index sets select.
// Both count exceedances against the identity split evaluated by their own code, as the
// efficient test does: p = (1 + #{b < B : stat*_b >= stat_B}) / (1 + B).
#include "common.h"

namespace et {

// ------------------------------------------------------------------ standard test
// Row map of split b: pooled items of x* in increasing order, then those of y* -- the
// index sets i*_x, i*_y of Alg. 4 -- so that staging through the map reads X* and Y*.
// One workgroup per split; maps k >= count are the identity (the observed split).
// Every member word holds exactly nx members (selection sampling); the index guards keep
// the writes inside the map whatever the words hold.
__global__ void __launch_bounds__(256) k_rowmap(const uint32_t* __restrict__ words, int64_t count,
                                                int64_t n, int64_t nx,
                                                int32_t* __restrict__ rowmap) {
  __shared__ int32_t scan[256];
  const int64_t b = blockIdx.x;
  int32_t* map = rowmap + b * n;
  const int tid = threadIdx.x;
  if (b >= count) {
    for (int64_t t = tid; t < n; t += 256) map[t] = (int32_t)t;
    return;
  }
  const int64_t W = (n + 31) / 32;
  const uint32_t* z = words + b * W;
  int64_t base = 0;  // x* members in the words before the current run of 256
  for (int64_t w0 = 0; w0 < W; w0 += 256) {
    const int64_t w = w0 + tid;
    uint32_t word = w < W ? z[w] : 0u;
    if (w == W - 1 && (n & 31)) word &= (1u << (n & 31)) - 1u;
    const int c = __popc(word);
    scan[tid] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the member counts
      const int v = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    int64_t xr = base + scan[tid] - c;  // members before item 32 w
    const int64_t run = scan[255];
    __syncthreads();
    if (w < W) {
      for (int k = 0; k < 32; ++k) {
        const int64_t t = w * 32 + k;
        if (t >= n) break;
        if ((word >> k) & 1u) {
          if (xr < nx) map[xr] = (int32_t)t;
          ++xr;
        } else {
          const int64_t yr = t - xr;  // y* items before t
          if (yr < n - nx) map[nx + yr] = (int32_t)t;
        }
      }
    }
    base += run;
  }
}

// Statistic of each recomputed test (its observed statistic, eq. 1 / eq. 2) into the list
// of split statistics; the identity split's refined-pair count; non-finite input.
__global__ void k_collect(const TestDesc* __restrict__ descs, int m, int64_t c0, int64_t B,
                          double* __restrict__ stats, int32_t* __restrict__ flags) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const TestDesc& d = descs[k];
  stats[c0 + k] = d.obs[3];
  if (d.flags[0]) atomicOr(&flags[0], 1);
  if (c0 + k == B) flags[1] = d.flags[1];
}

// Threshold (the identity split, stats[B]), exceedance count and p-value; copies the drawn
// splits' statistics to perm_out when given and the input was finite.
__global__ void __launch_bounds__(1024) k_count(const double* __restrict__ stats, int64_t B,
                                                const int32_t* __restrict__ flags,
                                                double* __restrict__ perm_out,
                                                DevResult* __restrict__ result) {
  __shared__ int64_t red[1024];
  const int tid = threadIdx.x;
  const double thr = stats[B];
  const bool bad = flags[0] != 0;
  int64_t c = 0;
  for (int64_t b = tid; b < B; b += 1024) {
    const double v = stats[b];
    c += v >= thr ? 1 : 0;
    if (perm_out && !bad) perm_out[b] = v;
  }
  red[tid] = c;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    DevResult r;
    r.statistic = thr;
    r.threshold = thr;
    r.count_ge = red[0];
    r.B = B;
    r.p_value = (1.0 + (double)red[0]) / (1.0 + (double)B);
    r.n_refined = flags[1];
    r.status = bad ? 2 : 0;
    r.pad = 0;
    if (bad) {
      r.statistic = __builtin_nan("");
      r.threshold = __builtin_nan("");
      r.p_value = __builtin_nan("");
    }
    *result = r;
  }
}

// ------------------------------------------------------------ pre-computation test
// The stored upper tiles of the pooled Gram are the pooled matrix D_WW (each unordered
// pair once; diagonal tiles in full).  For split z (bit 1 = x*), with row sums over the
// tile's x* columns s_x and y* columns s_y, the three block sums of the split are
//   off-diagonal tile: row in x*: W_xx += 2 s_x, W_xy += s_y;  row in y*: W_xy += s_x,
//                      W_yy += 2 s_y   (each entry stands for (a, b) and (b, a));
//   diagonal tile:     row in x*: W_xx += s_x, W_xy += s_y;    row in y*: W_yy += s_y
//                      (the tile holds both orders; x*-y* pairs are taken once).
// With the dense pooled matrix (Alg. 5 as printed: every tile of the nt x nt grid, D_YX
// included) every tile holds both orders of its pairs and takes the diagonal-tile rule: the
// X*X*, Y*Y* and X*Y* sub-blocks are read entry by entry and the Y*X* entries are skipped.
// Padding entries are 0.  One wave per (tile, 32-row strip, 64 splits): the strip sits in
// LDS and every lane (one split) reads the same entry, selects it by its own column bit and
// adds it in FP64.  No matrix product: this is the per-split extraction of Alg. 5.
// The strip is held in LDS as FP64 (the stored FP32 entries converted once).  An entry is
// selected by a fused multiply-add with the lane's column bit as 0.0 or 1.0, which adds it
// exactly or leaves the sum as it is; the bits, fixed for the whole strip, are converted
// once, so each entry costs one FMA.
template <typename T>
__global__ void __launch_bounds__(64) k_precomp(const TestDesc* __restrict__ descs,
                                                double* __restrict__ part, int64_t sg) {
  __shared__ double Ds[PC_ROWS * TILE];
  __shared__ double half_tot[PC_ROWS][2];
  const TestDesc d = descs[0];
  const int64_t g = blockIdx.x % sg;  // group of 64 split columns
  const int64_t u = blockIdx.x / sg;  // strip u: tile u / PC_STRIPS, rows 32 (u % PC_STRIPS) ..
  const int t = (int)(u / PC_STRIPS), h = (int)(u % PC_STRIPS);
  int i, j;
  if (d.dense) {
    i = t / d.nt;
    j = t % d.nt;
  } else {
    tile_coords(t, d.nt, &i, &j);
  }
  const int lane = threadIdx.x;
  {  // the 32 x 128 strip: every 16-byte load of the lane in flight before the LDS stores
    const uint4* src = (const uint4*)((const T*)d.D + (int64_t)t * TILE * TILE +
                                      (int64_t)h * PC_ROWS * TILE);
    constexpr int PER = 16 / sizeof(T);                  // entries per load
    constexpr int NLD = PC_ROWS * TILE / PER / 64;       // loads per lane
    uint4 v[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) v[k] = src[lane + 64 * k];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const T* e = (const T*)&v[k];
#pragma unroll
      for (int q = 0; q < PER; ++q) Ds[(lane + 64 * k) * PER + q] = (double)e[q];
    }
  }
  __syncthreads();
  {  // row totals of the strip, two lanes per row, fixed order
    const int r = lane >> 1, hf = lane & 1;
    double s = 0.0;
    for (int c = 0; c < TILE / 2; ++c) s += Ds[r * TILE + hf * (TILE / 2) + c];
    half_tot[r][hf] = s;
  }
  __syncthreads();
  const int64_t s = g * 64 + lane;  // < B_pad: Z columns past B hold no members
  uint32_t zc[TILE_WORDS];
#pragma unroll
  for (int q = 0; q < TILE_WORDS; ++q) zc[q] = d.Z[(int64_t)(j * TILE_WORDS + q) * d.B_pad + s];
  const uint32_t zr = d.Z[(int64_t)(i * TILE_WORDS + h) * d.B_pad + s];
  // a tile holding both orders of its pairs: a diagonal tile, or any tile of the dense matrix
  const bool both_orders = d.dense || i == j;
  double wxx = 0.0, wyy = 0.0, wxy = 0.0;
  for (int r = 0; r < PC_ROWS; ++r) {
    const double* row = Ds + r * TILE;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < TILE; ++c)
      a[c & 3] = fma(row[c], (double)((zc[c >> 5] >> (c & 31)) & 1u), a[c & 3]);
    const double sx = (a[0] + a[1]) + (a[2] + a[3]);
    const double sy = (half_tot[r][0] + half_tot[r][1]) - sx;
    const bool member = (zr >> r) & 1u;
    if (both_orders) {
      if (member) {
        wxx += sx;
        wxy += sy;
      } else {
        wyy += sy;
      }
    } else if (member) {
      wxx += 2.0 * sx;
      wxy += sy;
    } else {
      wxy += sx;
      wyy += 2.0 * sy;
    }
  }
  if (s <= d.B) {
    part[(u * 3 + 0) * d.B_pad + s] = wxx;
    part[(u * 3 + 1) * d.B_pad + s] = wyy;
    part[(u * 3 + 2) * d.B_pad + s] = wxy;
  }
}

struct Csum2 {  // Neumaier-compensated sum
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

// Statistics of 64 split columns per workgroup: 16 groups of waves each take every 16th
// strip (compensated sums), then wave 0 adds the 16 group sums in order.
constexpr int PCS_GROUPS = 16;
__global__ void __launch_bounds__(64 * PCS_GROUPS) k_precomp_stat(const TestDesc* __restrict__ descs,
                                                                  const double* __restrict__ part,
                                                                  int64_t nstrips,
                                                                  double* __restrict__ stats) {
  __shared__ double red[3][PCS_GROUPS][64];
  const TestDesc d = descs[0];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t s = (int64_t)blockIdx.x * 64 + c;  // < B_pad
  Csum2 acc[3];
  for (int64_t u = g; u < nstrips; u += PCS_GROUPS)
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k].add(part[(u * 3 + k) * d.B_pad + s]);
#pragma unroll
  for (int k = 0; k < 3; ++k) red[k][g][c] = acc[k].value();
  __syncthreads();
  if (g != 0 || s > d.B) return;
  Csum2 w[3];
  for (int q = 0; q < PCS_GROUPS; ++q)
#pragma unroll
    for (int k = 0; k < 3; ++k) w[k].add(red[k][q][c]);
  const double nx = d.nx, ny = d.ny;
  const double txx = w[0].value() / (nx * nx), tyy = w[1].value() / (ny * ny);
  const double txy = 2.0 * w[2].value() / (nx * ny);
  stats[s] = d.kind == KIND_ED ? (txy - txx) - tyy : (txx + tyy) - txy;
}

// ------------------------------------------------------------------- launchers
void launch_rowmap(const uint32_t* words, int64_t count, int64_t maps, int64_t n, int64_t nx,
                   int32_t* rowmap, hipStream_t st) {
  if (maps > 0)
    hipLaunchKernelGGL(k_rowmap, dim3((unsigned)maps), dim3(256), 0, st, words, count, n, nx,
                       rowmap);
}
void launch_collect(const TestDesc* d, int m, int64_t c0, int64_t B, double* stats,
                    int32_t* flags, hipStream_t st) {
  if (m > 0)
    hipLaunchKernelGGL(k_collect, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, d, m, c0, B,
                       stats, flags);
}
void launch_count(const double* stats, int64_t B, const int32_t* flags, double* perm_out,
                  DevResult* result, hipStream_t st) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(1024), 0, st, stats, B, flags, perm_out, result);
}
// Strip sums of every split column: ntiles * PC_STRIPS strips x ceil((B + 1) / 64) groups.
void launch_precomp(bool f64, const TestDesc* d, int64_t ntiles, int64_t B, double* part,
                    hipStream_t st) {
  const int64_t sg = (B + 1 + 63) / 64;
  const int64_t blocks = ntiles * PC_STRIPS * sg;
  if (f64)
    hipLaunchKernelGGL(k_precomp<double>, dim3((unsigned)blocks), dim3(64), 0, st, d, part, sg);
  else
    hipLaunchKernelGGL(k_precomp<float>, dim3((unsigned)blocks), dim3(64), 0, st, d, part, sg);
}
void launch_precomp_stat(const TestDesc* d, int64_t ntiles, int64_t B, const double* part,
                         double* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_precomp_stat, dim3((unsigned)((B + 1 + 63) / 64)), dim3(64 * PCS_GROUPS), 0,
                     st, d, part, ntiles * PC_STRIPS, stats);
}

}  // namespace et
