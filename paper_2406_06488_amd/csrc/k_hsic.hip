// HSIC independence permutation test (the extension proposed in the paper's discussion):
// paired samples (x_i, y_i), i < n; Gaussian kernel matrices K of x and L of y are
// computed once (the staging and Gram kernels of the two-sample test, one "sample" each);
// each permutation pi of the y sample then costs one pass over the n^2 entries:
//   Kt = K - diag(K), Lt = L - diag(L), r = Kt 1, s = Lt 1,
//   T1(pi) = sum_{i,j} Kt[i][j] Lt[pi_i][pi_j],  T3(pi) = sum_i r_i s_{pi_i},
//   T2 = (1^T Kt 1)(1^T Lt 1),
//   HSIC(pi) = [T1 + T2 / ((n-1)(n-2)) - 2 T3 / (n-2)] / (n (n-3))
// (the unbiased estimator of Song et al. 2012).  Unlike the two-sample statistics, T1 is
// not a quadratic form in a 0/1 vector, so no contraction shortens it: each permutation
// gathers n^2 entries of Lt, the cost the discussion anticipates.
#include "common.h"

namespace et {

// ------------------------------------------------------------------ permutations
// Permutation b of 0..n-1: items ordered by a 64-bit Philox4x32-10 key, key (seed_lo,
// seed_hi), counter (t/2, b_lo, b_hi, 1) (even t: words 0, 1; odd t: words 2, 3; low word
// first), ties by index.  One workgroup per permutation: a bitonic sort of (key, item) in
// LDS over the next power of two (padding keys all ones, padding items >= n, so they sort
// after every real item).  perms[q][i] = the item placed at position i, for b = b0 + q with
// q < count; slots count .. total - 1 hold the identity.
__device__ inline uint64_t perm_key(uint32_t k0, uint32_t k1, uint32_t b_lo, uint32_t b_hi,
                                    uint32_t t) {
  const uint4 r = philox4x32_10(make_uint4(t >> 1, b_lo, b_hi, 1u), k0, k1);
  return (t & 1u) ? ((uint64_t)r.w << 32) | r.z : ((uint64_t)r.y << 32) | r.x;
}

__global__ void __launch_bounds__(1024) k_permgen(int64_t n, uint64_t seed, int64_t b0,
                                                  int64_t count, int32_t* __restrict__ perms) {
  __shared__ uint64_t key[HSIC_NMAX];
  __shared__ int32_t item[HSIC_NMAX];
  const int64_t q = blockIdx.x;
  int32_t* out = perms + q * n;
  const int tid = threadIdx.x;
  if (q >= count) {
    for (int64_t t = tid; t < n; t += 1024) out[t] = (int32_t)t;
    return;
  }
  const uint64_t b = (uint64_t)(b0 + q);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int t = tid; t < n2; t += 1024) {
    key[t] = t < n ? perm_key(k0, k1, (uint32_t)b, (uint32_t)(b >> 32), (uint32_t)t) : ~0ull;
    item[t] = t;
  }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < n2; t += 1024) {
        const int l = t ^ j;
        if (l > t) {
          const bool ascending = (t & k) == 0;
          const uint64_t kt = key[t], kl = key[l];
          const int32_t it = item[t], il = item[l];
          const bool greater = kt > kl || (kt == kl && it > il);
          if (greater == ascending) {
            key[t] = kl;
            key[l] = kt;
            item[t] = il;
            item[l] = it;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int64_t t = tid; t < n; t += 1024) out[t] = item[t];
}

// ------------------------------------------------------------------ kernel matrices
// Dense Kt and Lt (row-major n x n, zero diagonal) from the stored upper tiles of the two
// one-sample Grams (descs[0]: x, descs[1]: y; blockIdx.y picks the matrix).
template <typename T>
__global__ void __launch_bounds__(256) k_hsic_unpack(const TestDesc* __restrict__ descs, int64_t n,
                                                     T* __restrict__ kx, T* __restrict__ ky) {
  const TestDesc& d = descs[blockIdx.y];
  T* out = blockIdx.y == 0 ? kx : ky;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int64_t a = e / n, c = e % n;
  if (a == c) {
    out[e] = (T)0;
    return;
  }
  int i = (int)(a / TILE), j = (int)(c / TILE), r = (int)(a % TILE), col = (int)(c % TILE);
  if (i > j) {
    int s = i; i = j; j = s;
    s = r; r = col; col = s;
  }
  out[e] = ((const T*)d.D)[(int64_t)tile_index(i, j, d.nt) * TILE * TILE + r * TILE + col];
}

// Row sums r = Kt 1 and s = Lt 1 in FP64: one wave per row (blockIdx.y picks the matrix),
// lane-strided partial sums combined by a fixed butterfly.
template <typename T>
__global__ void __launch_bounds__(256) k_hsic_rows(const T* __restrict__ kx,
                                                   const T* __restrict__ ky, int64_t n,
                                                   double* __restrict__ rx,
                                                   double* __restrict__ ry) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const T* src = (blockIdx.y == 0 ? kx : ky) + row * n;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s += (double)src[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) (blockIdx.y == 0 ? rx : ry)[row] = s;
}

struct Hsum {  // Neumaier-compensated sum
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

// 1^T Kt 1 and 1^T Lt 1 (hs[0], hs[1]); the two staging flags merged for the count
// (flags[0]: non-finite input in x or y; flags[1]: refined pairs of both Grams).
__global__ void __launch_bounds__(256) k_hsic_sums(const double* __restrict__ rx,
                                                   const double* __restrict__ ry, int64_t n,
                                                   const TestDesc* __restrict__ descs,
                                                   double* __restrict__ hs,
                                                   int32_t* __restrict__ flags) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  Hsum a, b;
  for (int64_t i = tid; i < n; i += 256) {
    a.add(rx[i]);
    b.add(ry[i]);
  }
  red[0][tid] = a.value();
  red[1][tid] = b.value();
  __syncthreads();
  if (tid < 2) {
    Hsum t;
    for (int k = 0; k < 256; ++k) t.add(red[tid][k]);
    hs[tid] = t.value();
  }
  if (tid == 2) {
    flags[0] = (descs[0].flags[0] | descs[1].flags[0]) ? 1 : 0;
    flags[1] = descs[0].flags[1] + descs[1].flags[1];
  }
}

// ------------------------------------------------------------------ permutations' terms
// T1 and T3 of permutation b over a block of HSIC_RB rows of Kt: for each row i, row pi_i of
// Lt goes to LDS (coalesced), then every lane sums Kt[i][j] * Lt[pi_i][pi_j] over its
// columns j (at most HSIC_NMAX / 256 terms; the products of two FP32 entries are exact in
// FP64) and adds that row sum to a compensated accumulator.  The three terms of the
// estimator cancel to a small fraction of their size, so T1 is kept to about one rounding
// of itself.  The workgroup's compensated partials, combined in a fixed order, go to
// part[(b * nblk + blk) * 2 + {0, 1}].
template <typename T>
__global__ void __launch_bounds__(256) k_hsic_terms(const T* __restrict__ kx,
                                                    const T* __restrict__ ky, int64_t n,
                                                    const int32_t* __restrict__ perms,
                                                    const double* __restrict__ rx,
                                                    const double* __restrict__ ry, int64_t nblk,
                                                    double* __restrict__ part) {
  __shared__ T lrow[HSIC_NMAX];
  __shared__ double red[256][2];
  // Work unit u = blk * nperm + b, numbered so that each XCD takes runs of consecutive units:
  // a run covers one row block for several permutations, whose Kt rows its L2 then serves.
  const int64_t nperm = gridDim.x / nblk;
  const int64_t u = xcd_grouped(blockIdx.x, gridDim.x);
  const int64_t blk = u / nperm, b = u % nperm;
  const int32_t* pi = perms + b * n;
  const int tid = threadIdx.x;
  constexpr int PER = HSIC_NMAX / 256;
  int32_t pj[PER];  // pi_j of the lane's columns j = tid + 256 k (fixed for the workgroup)
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t j = tid + 256 * k;
    pj[k] = j < n ? pi[j] : 0;
  }
  Hsum acc;
  double t3 = 0.0;
  const int64_t i0 = blk * HSIC_RB;
  for (int r = 0; r < HSIC_RB; ++r) {
    const int64_t i = i0 + r;
    if (i >= n) break;
    const int64_t pii = pi[i];
    __syncthreads();
    for (int64_t j = tid; j < n; j += 256) lrow[j] = ky[pii * n + j];
    __syncthreads();
    const T* krow = kx + i * n;
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int64_t j = tid + 256 * k;
      if (j < n) rs = fma((double)krow[j], (double)lrow[pj[k]], rs);
    }
    acc.add(rs);
    if (tid == 0) t3 = fma(rx[i], ry[pii], t3);
  }
  red[tid][0] = acc.s;
  red[tid][1] = acc.c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {  // compensated pairwise combination, fixed tree
    if (tid < s) {
      Hsum u;
      u.s = red[tid][0];
      u.c = red[tid][1] + red[tid + s][1];
      u.add(red[tid + s][0]);
      red[tid][0] = u.s;
      red[tid][1] = u.c;
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[(b * nblk + blk) * 2] = red[0][0] + red[0][1];
    part[(b * nblk + blk) * 2 + 1] = t3;
  }
}

// HSIC of 64 permutations per workgroup from their row-block partials: 16 groups of waves
// each take every 16th block (compensated), then wave 0 adds the 16 group sums in order.
constexpr int HS_GROUPS = 16;
__global__ void __launch_bounds__(64 * HS_GROUPS) k_hsic_stat(const double* __restrict__ part,
                                                              int64_t nblk, int64_t nperm,
                                                              int64_t n,
                                                              const double* __restrict__ hs,
                                                              double* __restrict__ stats) {
  __shared__ double red[2][HS_GROUPS][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 64 + c;
  Hsum t1, t3;
  if (b < nperm)
    for (int64_t k = g; k < nblk; k += HS_GROUPS) {
      t1.add(part[(b * nblk + k) * 2]);
      t3.add(part[(b * nblk + k) * 2 + 1]);
    }
  red[0][g][c] = t1.value();
  red[1][g][c] = t3.value();
  __syncthreads();
  if (g != 0 || b >= nperm) return;
  Hsum u1, u3;
  for (int q = 0; q < HS_GROUPS; ++q) {
    u1.add(red[0][q][c]);
    u3.add(red[1][q][c]);
  }
  const double dn = (double)n;
  const double t2 = hs[0] * hs[1];
  stats[b] = (u1.value() + t2 / ((dn - 1.0) * (dn - 2.0)) - 2.0 * u3.value() / (dn - 2.0)) /
             (dn * (dn - 3.0));
}

// ------------------------------------------------------------------- launchers
void launch_permgen(int64_t n, uint64_t seed, int64_t b0, int64_t count, int64_t total,
                    int32_t* perms, hipStream_t st) {
  if (total > 0)
    hipLaunchKernelGGL(k_permgen, dim3((unsigned)total), dim3(1024), 0, st, n, seed, b0, count,
                       perms);
}
void launch_hsic_prep(bool f64, const TestDesc* d, int64_t n, void* kx, void* ky, double* rx,
                      double* ry, double* hs, int32_t* flags, hipStream_t st) {
  const dim3 gu((unsigned)((n * n + 255) / 256), 2), gr((unsigned)((n + 3) / 4), 2);
  if (f64) {
    hipLaunchKernelGGL(k_hsic_unpack<double>, gu, dim3(256), 0, st, d, n, (double*)kx, (double*)ky);
    hipLaunchKernelGGL(k_hsic_rows<double>, gr, dim3(256), 0, st, (const double*)kx,
                       (const double*)ky, n, rx, ry);
  } else {
    hipLaunchKernelGGL(k_hsic_unpack<float>, gu, dim3(256), 0, st, d, n, (float*)kx, (float*)ky);
    hipLaunchKernelGGL(k_hsic_rows<float>, gr, dim3(256), 0, st, (const float*)kx,
                       (const float*)ky, n, rx, ry);
  }
  hipLaunchKernelGGL(k_hsic_sums, dim3(1), dim3(256), 0, st, rx, ry, n, d, hs, flags);
}
void launch_hsic_terms(bool f64, const void* kx, const void* ky, int64_t n, const int32_t* perms,
                       int64_t nperm, const double* rx, const double* ry, double* part,
                       hipStream_t st) {
  const int64_t nblk = (n + HSIC_RB - 1) / HSIC_RB;
  const dim3 g((unsigned)(nperm * nblk));
  if (f64)
    hipLaunchKernelGGL(k_hsic_terms<double>, g, dim3(256), 0, st, (const double*)kx,
                       (const double*)ky, n, perms, rx, ry, nblk, part);
  else
    hipLaunchKernelGGL(k_hsic_terms<float>, g, dim3(256), 0, st, (const float*)kx,
                       (const float*)ky, n, perms, rx, ry, nblk, part);
}
void launch_hsic_stat(const double* part, int64_t n, int64_t nperm, const double* hs,
                      double* stats, hipStream_t st) {
  const int64_t nblk = (n + HSIC_RB - 1) / HSIC_RB;
  hipLaunchKernelGGL(k_hsic_stat, dim3((unsigned)((nperm + 63) / 64)), dim3(64 * HS_GROUPS), 0, st,
                     part, nblk, nperm, n, hs, stats);
}

}  // namespace et
