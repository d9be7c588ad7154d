// Input staging: column means of the pooled sample, centred + cast operand rows,
// squared row norms and the non-finite check.
//
// Distances are invariant to a common translation of X and Y, so subtracting
// the pooled column mean changes no block entry in exact arithmetic; it keeps
// |x|^2 + |y|^2 - 2 x.y from cancelling when the data sit far from the origin.
// The FP64 form stages the data unchanged (its blocks use direct differences).
#include "common.h"

namespace et {

constexpr int ROWCHUNK = COLSUM_ROWS;

__device__ inline float load_in_f32(const TestDesc& d, int64_t t, int k) {
  return pooled_row<float>(d, t)[k];
}
__device__ inline double load_in_f64(const TestDesc& d, int64_t t, int k) {
  return pooled_row<double>(d, t)[k];
}

// Partial column sums over chunks of ROWCHUNK pooled rows (FP64).  All ROWCHUNK loads of a
// thread are issued before the (fixed-order) sum, so they are in flight together.  Tests
// whose Gram reads fp16 pairs also take max |x| over the input (one atomic per workgroup),
// which sets the scale of those pairs.
__global__ void __launch_bounds__(256) k_colpart(const TestDesc* __restrict__ descs,
                                                 const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  const int cpw = colpart_chunks_per_wg(d.p);
  int rc, k;
  bool ok;
  if (cpw > 1) {  // p < 256: row chunks local * cpw + threadIdx.x / p, all p columns
    const int sub = (int)threadIdx.x / d.p;
    k = (int)threadIdx.x % d.p;
    rc = (int)(local * cpw) + sub;
    ok = sub < cpw && rc < d.nrowchunks;
  } else {
    const int ncb = (d.p + 255) / 256;
    rc = (int)(local / ncb);
    k = (int)(local % ncb) * 256 + threadIdx.x;
    ok = k < d.p;
  }
  const int64_t n = (int64_t)d.nx + d.ny;
  const int64_t t0 = (int64_t)rc * ROWCHUNK;
  float v[ROWCHUNK];
#pragma unroll
  for (int r = 0; r < ROWCHUNK; ++r) v[r] = ok && t0 + r < n ? load_in_f32(d, t0 + r, k) : 0.0f;
  double s = 0.0;
  float mx = 0.0f;
#pragma unroll
  for (int r = 0; r < ROWCHUNK; ++r) {
    s += (double)v[r];
    mx = fmaxf(mx, fabsf(v[r]));  // fmaxf drops NaN; an Inf makes the scale 1 (flagged anyway)
  }
  if (ok) d.colpart[(int64_t)rc * d.p + k] = s;
  if (d.gop == GOP_F16PAIR) {  // uniform per workgroup: one atomic per workgroup
    __shared__ float wmax[4];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) mx = fmaxf(mx, __shfl_xor(mx, m, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      mx = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
      // non-negative floats order like their bit patterns
      if (mx > 0.0f) atomicMax((unsigned int*)&d.flags[FLAG_XMAX], __float_as_uint(mx));
    }
  }
}

// Column means: 64 columns per workgroup, 16 groups of waves each summing every 16th
// partial, then the 16 group sums in order (a fixed order: the result is reproducible).
__global__ void __launch_bounds__(64 * CM_GROUPS) k_colmean(const TestDesc* __restrict__ descs,
                                                            const int64_t* __restrict__ offs,
                                                            int ntests) {
  __shared__ double red[CM_GROUPS][64];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int k = (int)(blockIdx.x - offs[ti]) * 64 + c;
  double s = 0.0;
  if (k < d.p)
    for (int rc = g; rc < d.nrowchunks; rc += CM_GROUPS) s += d.colpart[(int64_t)rc * d.p + k];
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && k < d.p) {
    double t = 0.0;
    for (int q = 0; q < CM_GROUPS; ++q) t += red[q][c];
    d.colmean[k] = t / (double)((int64_t)d.nx + d.ny);
  }
}

// fp16-pair operands: w -> (hi, lo) with hi = fp16(w 2^e), lo = fp16(w 2^e - hi), returned
// packed (hi in the low half; the staging writes them to two planes); *r = (hi + lo) 2^-e, the value the Gram's products see (its norm goes to nrm, so
// that |a|^2 + |b|^2 - 2 g is formed from one set of operand values).
__device__ inline uint32_t f16_pair(float w, int e, double* r) {
  const float hs = ldexpf(w, e);
  const _Float16 hi = (_Float16)hs;
  const _Float16 lo = (_Float16)(hs - (float)hi);  // the difference is exact in FP32
  *r = ldexp((double)(float)hi + (double)(float)lo, -e);
  return (uint32_t)__builtin_bit_cast(uint16_t, hi) |
         ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
}

// Sum over the lpr lanes (a power of two) that stage one row.
__device__ inline double row_sum(double v, int lpr) {
  for (int off = lpr >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// lpr = stage_lanes_per_row(p_pad) lanes per padded pooled row (a whole wave from
// p_pad = 256 on): write W[pos][0..p_pad), nrm[pos]; flag NaN/Inf.
__global__ void __launch_bounds__(256) k_stage(const TestDesc* __restrict__ descs,
                                               const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  const int lpr = stage_lanes_per_row(d.p_pad);
  const int lane = (threadIdx.x & 63) & (lpr - 1);  // lane within the row's group
  const int64_t pos = (local * 4 + (threadIdx.x >> 6)) * (64 / lpr) + (threadIdx.x & 63) / lpr;
  const bool live = pos < (int64_t)d.nt * TILE;
  const int64_t split = (int64_t)d.tx * TILE;
  int64_t t = -1;  // pooled input row, -1 for padding
  if (pos < split) {
    if (pos < d.nx) t = pos;
  } else {
    const int64_t yi = pos - split;
    if (yi < d.ny) t = d.nx + yi;
  }
  bool bad = false;
  double nrm = 0.0;
  if (d.gop == GOP_F64) {
    double* W = (double*)d.W + pos * d.p_pad;
    for (int k = lane; k < d.p_pad; k += lpr) {
      double v = 0.0;
      if (t >= 0 && k < d.p) {
        v = load_in_f64(d, t, k);
        bad |= !isfinite(v);
      }
      if (live) W[k] = v;
      nrm += v * v;
    }
    nrm = row_sum(nrm, lpr);
    if (lane == 0 && live) ((double*)d.nrm)[pos] = nrm;
  } else {
    const bool bf = d.gop == GOP_BF16;
    const int e = bf ? 0 : f16_split_exponent(d);
    // K-blocked 16-bit operands: BF16 value k at (chunk k / 32, slot k % 32); fp16 pair k
    // hi at (chunk k / 16, slot k % 16), lo at slot 16 + k % 16
    uint16_t* Wu = (uint16_t*)d.W;
    const int64_t nch = d.p_pad / chunk_coords(d.gop);
    const float* src = t < 0 ? nullptr : pooled_row<float>(d, t);
    // four columns per lane when every row starts on a 16-byte boundary
    const bool vec = (d.p & 3) == 0 && (((uintptr_t)d.X | (uintptr_t)d.Y) & 15) == 0;
    if (vec) {
      for (int k = 4 * lane; k < d.p_pad; k += 4 * lpr) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (src && k < d.p) {
          const float4 x = *(const float4*)(src + k);
          bad |= !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(x.w));
          v.x = (float)((double)x.x - d.colmean[k]);
          v.y = (float)((double)x.y - d.colmean[k + 1]);
          v.z = (float)((double)x.z - d.colmean[k + 2]);
          v.w = (float)((double)x.w - d.colmean[k + 3]);
        }
        if (bf) {
          const uint16_t h0 = f32_to_bf16_rn(v.x), h1 = f32_to_bf16_rn(v.y);
          const uint16_t h2 = f32_to_bf16_rn(v.z), h3 = f32_to_bf16_rn(v.w);
          uint2 o;
          o.x = (uint32_t)h0 | ((uint32_t)h1 << 16);
          o.y = (uint32_t)h2 | ((uint32_t)h3 << 16);
          if (live) *(uint2*)(Wu + blocked_index(pos, k >> 5, k & 31, nch)) = o;
          const double r0 = bf16_to_f32(h0), r1 = bf16_to_f32(h1);
          const double r2 = bf16_to_f32(h2), r3 = bf16_to_f32(h3);
          nrm += ((r0 * r0 + r1 * r1) + r2 * r2) + r3 * r3;
        } else {
          double r0, r1, r2, r3;
          const uint32_t q0 = f16_pair(v.x, e, &r0), q1 = f16_pair(v.y, e, &r1);
          const uint32_t q2 = f16_pair(v.z, e, &r2), q3 = f16_pair(v.w, e, &r3);
          uint2 hi, lo;  // the hi plane and the lo plane, four halves each
          hi.x = (q0 & 0xFFFFu) | (q1 << 16);
          hi.y = (q2 & 0xFFFFu) | (q3 << 16);
          lo.x = (q0 >> 16) | (q1 & 0xFFFF0000u);
          lo.y = (q2 >> 16) | (q3 & 0xFFFF0000u);
          uint16_t* wp = Wu + blocked_index(pos, k >> 4, k & 15, nch);
          if (live) {
            *(uint2*)wp = hi;
            *(uint2*)(wp + 16) = lo;
          }
          nrm += ((r0 * r0 + r1 * r1) + r2 * r2) + r3 * r3;
        }
      }
    } else {
      for (int k = lane; k < d.p_pad; k += lpr) {
        float v = 0.0f;
        if (src && k < d.p) {
          const float x = src[k];
          bad |= !isfinite(x);
          v = (float)((double)x - d.colmean[k]);
        }
        if (bf) {
          const uint16_t h = f32_to_bf16_rn(v);
          if (live) Wu[blocked_index(pos, k >> 5, k & 31, nch)] = h;
          const float r = bf16_to_f32(h);
          nrm += (double)r * (double)r;
        } else {
          double r;
          const uint32_t q = f16_pair(v, e, &r);
          uint16_t* wp = Wu + blocked_index(pos, k >> 4, k & 15, nch);
          if (live) {
            wp[0] = (uint16_t)(q & 0xFFFFu);
            wp[16] = (uint16_t)(q >> 16);
          }
          nrm += r * r;
        }
      }
    }
    nrm = row_sum(nrm, lpr);
    if (lane == 0 && live) ((float*)d.nrm)[pos] = (float)nrm;
  }
  if (bad) {
    atomicOr(&d.flags[0], 1);
    if (d.pflags) atomicOr(&d.pflags[0], 1);  // the MMD test fed by this staging
  }
}

// Clear the per-test flag words (a kernel rather than a memset so that the
// launch sequence can be captured into a graph).  With a prefix table, only
// tests that own workgroups in it are cleared.
__global__ void k_clear_flags(const TestDesc* __restrict__ descs, const int64_t* __restrict__ offs,
                              int ntests) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntests && (offs == nullptr || offs[t + 1] > offs[t])) {
    for (int k = 0; k < FLAG_WORDS; ++k) descs[t].flags[k] = 0;
  }
}

void launch_clear_flags(hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  hipLaunchKernelGGL(k_clear_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, offs, n);
}
void launch_colpart(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_colpart, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}
void launch_colmean(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0)
    hipLaunchKernelGGL(k_colmean, dim3((unsigned)blocks), dim3(64 * CM_GROUPS), 0, st, d, offs, n);
}
void launch_stage(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_stage, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}

}  // namespace et
