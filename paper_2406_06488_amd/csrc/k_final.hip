// Resampled statistics, threshold, exceedance count and p-value.
//
//   stat*_c = sign * (1/nx + 1/ny)^2 * 2 * sum over row ranges of part[., c]
// (sign -1 for energy distance, +1 for MMD; the factor 2 undoes the halved
// diagonal tiles).  Column B is the identity split: its value is the counting
// threshold, so a resampled split equal to the observed one always counts.
// p = (1 + #{b < B : stat*_b >= threshold}) / (1 + B)  (Section 3.1).
#include "common.h"

namespace et {

// One workgroup per 64 split columns: 16 groups of waves each sum every 16th row range,
// then wave 0 adds the 16 group sums in order.  Every workgroup also evaluates the
// identity column B with the same loads in the same order, so all of them hold the
// threshold bit for bit as the column's own workgroup computes it.  Exceedances are
// counted with one integer atomic per workgroup; the last workgroup of a test writes the
// result.

__device__ inline double split_statistic(const TestDesc& d, double q) {
  if (d.prec != PREC_F64) q /= d.obs[5];  // undo the power-of-two scale of the fp16 planes
  const double a = 1.0 / d.nx + 1.0 / d.ny;
  const double coef = a * a * 2.0;
  return d.kind == KIND_ED ? -coef * q : coef * q;
}

__global__ void __launch_bounds__(64 * PS_GROUPS) k_pstat(const TestDesc* __restrict__ descs,
                                                          const int64_t* __restrict__ offs,
                                                          int ntests) {
  __shared__ double red[PS_GROUPS][65];  // [.][64]: the identity column
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t wg = blockIdx.x - offs[ti];
  const int64_t nwg = offs[ti + 1] - offs[ti];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t col = wg * 64 + c;
  double s = 0.0;
  for (int rk = g; rk < d.n_rowk; rk += PS_GROUPS) s += d.part[(int64_t)rk * d.B_pad + col];
  red[g][c] = s;
  if (c == 0) {
    double sb = 0.0;
    for (int rk = g; rk < d.n_rowk; rk += PS_GROUPS) sb += d.part[(int64_t)rk * d.B_pad + d.B];
    red[g][64] = sb;
  }
  __syncthreads();
  if (g != 0) return;
  double q = 0.0, qb = 0.0;
  for (int k = 0; k < PS_GROUPS; ++k) {
    q += red[k][c];
    qb += red[k][64];
  }
  const double v = split_statistic(d, q), thr = split_statistic(d, qb);
  d.pstat[col] = v;
  const bool bad = d.flags[0] != 0 || d.flags[2] != 0;
  const bool drawn = col < d.B;
  if (drawn && d.perm_out && !bad) d.perm_out[col] = v;
  const uint64_t ge = __ballot(drawn && v >= thr);
  // one 64-bit atomic carries both the count (low 32 bits; B < 2^31) and the number of
  // finished workgroups (high 32 bits), so the last workgroup's returned value already
  // holds every other workgroup's count: no fence is needed
  unsigned long long* cnt = (unsigned long long*)(d.flags + FLAG_COUNT);
  if (c == 0) {
    const unsigned long long add = (1ull << 32) | (unsigned long long)__popcll(ge);
    const unsigned long long old = atomicAdd(cnt, add);
    if ((int64_t)(old >> 32) == nwg - 1) {
      const int64_t count = (int64_t)((old + add) & 0xFFFFFFFFull);
      DevResult r;
      r.statistic = d.obs[3];
      r.threshold = thr;
      r.count_ge = count;
      r.B = d.B;
      r.p_value = (1.0 + (double)count) / (1.0 + (double)d.B);
      r.n_refined = d.flags[1];
      r.status = d.flags[0] ? 2 : (d.flags[2] ? 1 : 0);
      r.pad = 0;
      if (bad) {
        r.statistic = __builtin_nan("");
        r.p_value = __builtin_nan("");
      }
      *d.result = r;
      if (d.out6) __builtin_memcpy(d.out6, &r, 6 * sizeof(double));
    }
  }
}

// Full row-major blocks from the stored tiles (for inspection of the block stage).
template <typename T>
__global__ void __launch_bounds__(256) k_unpack(const TestDesc* __restrict__ descs, T* dxx,
                                                T* dyy, T* dxy) {
  const TestDesc d = descs[0];
  const int64_t nxx = (int64_t)d.nx * d.nx, nyy = (int64_t)d.ny * d.ny,
                nxy = (int64_t)d.nx * d.ny;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const T* D = (const T*)d.D;
  int64_t a, b;
  int pa, pb;  // padded pooled positions
  T* out;
  if (e < nxx) {
    a = e / d.nx; b = e % d.nx; pa = (int)a; pb = (int)b; out = dxx + e;
  } else if (e < nxx + nyy) {
    const int64_t f = e - nxx;
    a = f / d.ny; b = f % d.ny;
    pa = d.tx * TILE + (int)a; pb = d.tx * TILE + (int)b; out = dyy + f;
  } else if (e < nxx + nyy + nxy) {
    const int64_t f = e - nxx - nyy;
    a = f / d.ny; b = f % d.ny;
    pa = (int)a; pb = d.tx * TILE + (int)b; out = dxy + f;
  } else {
    return;
  }
  int i = pa / TILE, j = pb / TILE, r = pa % TILE, c = pb % TILE;
  if (i > j) { int q = i; i = j; j = q; q = r; r = c; c = q; }
  *out = D[(int64_t)tile_index(i, j, d.nt) * TILE * TILE + r * TILE + c];
}

// Caller-supplied splits (public layout, words[q * W + t/32]) -> internal layout.
__global__ void __launch_bounds__(256) k_member_import(const TestDesc* __restrict__ descs,
                                                       const uint32_t* __restrict__ words) {
  const TestDesc d = descs[0];
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= d.B_pad) return;
  const int64_t n = (int64_t)d.nx + d.ny, W = (n + 31) / 32;
  const int xw = d.tx * TILE_WORDS, yw = d.ty * TILE_WORDS;
  int64_t members = 0;
  for (int w = 0; w < xw + yw; ++w) {
    uint32_t word = 0;
    for (int bit = 0; bit < 32; ++bit) {
      const int64_t pos = (int64_t)w * 32 + bit;
      int64_t t;  // pooled item at this padded position, -1 for padding
      if (w < xw) t = pos < d.nx ? pos : -1;
      else t = (pos - (int64_t)xw * 32) < d.ny ? d.nx + (pos - (int64_t)xw * 32) : -1;
      uint32_t v = 0;
      if (t >= 0) {
        if (col < d.B) v = (words[col * W + t / 32] >> (t % 32)) & 1u;
        else if (col == d.B) v = t < d.nx ? 1u : 0u;
      }
      word |= v << bit;
      members += v;
    }
    d.Z[(int64_t)w * d.B_pad + col] = word;
  }
  if (col < d.B && members != d.nx) atomicOr(&d.flags[2], 1);
}

void launch_pstat(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0)
    hipLaunchKernelGGL(k_pstat, dim3((unsigned)blocks), dim3(64 * PS_GROUPS), 0, st, d, offs, n);
}
void launch_unpack(bool f64, int64_t elems, hipStream_t st, const TestDesc* d, void* xx, void* yy,
                   void* xy) {
  const unsigned blocks = (unsigned)((elems + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(k_unpack<double>, dim3(blocks), dim3(256), 0, st, d, (double*)xx,
                       (double*)yy, (double*)xy);
  else
    hipLaunchKernelGGL(k_unpack<float>, dim3(blocks), dim3(256), 0, st, d, (float*)xx,
                       (float*)yy, (float*)xy);
}
void launch_member_import(int64_t bpad, hipStream_t st, const TestDesc* d, const uint32_t* w) {
  hipLaunchKernelGGL(k_member_import, dim3((unsigned)((bpad + 255) / 256)), dim3(256), 0, st, d, w);
}

}  // namespace et
