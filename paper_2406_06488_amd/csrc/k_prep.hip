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
  return t < d.nx ? ((const float*)d.X)[t * d.p + k] : ((const float*)d.Y)[(t - d.nx) * d.p + k];
}
__device__ inline double load_in_f64(const TestDesc& d, int64_t t, int k) {
  return t < d.nx ? ((const double*)d.X)[t * d.p + k] : ((const double*)d.Y)[(t - d.nx) * d.p + k];
}

// Partial column sums over chunks of ROWCHUNK pooled rows (FP64).
__global__ void __launch_bounds__(256) k_colpart(const TestDesc* __restrict__ descs,
                                                 const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  const int ncb = (d.p + 255) / 256;
  const int rc = (int)(local / ncb);
  const int k = (int)(local % ncb) * 256 + threadIdx.x;
  if (k >= d.p) return;
  const int64_t n = (int64_t)d.nx + d.ny;
  const int64_t t0 = (int64_t)rc * ROWCHUNK;
  const int64_t t1 = t0 + ROWCHUNK < n ? t0 + ROWCHUNK : n;
  // four independent running sums (rows t0 + 4i + r) keep several loads in flight
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t t = t0;
  for (; t + 4 <= t1; t += 4) {
    s0 += (double)load_in_f32(d, t, k);
    s1 += (double)load_in_f32(d, t + 1, k);
    s2 += (double)load_in_f32(d, t + 2, k);
    s3 += (double)load_in_f32(d, t + 3, k);
  }
  for (; t < t1; ++t) s0 += (double)load_in_f32(d, t, k);
  d.colpart[(int64_t)rc * d.p + k] = (s0 + s1) + (s2 + s3);
}

__global__ void __launch_bounds__(256) k_colmean(const TestDesc* __restrict__ descs,
                                                 const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int k = (int)(blockIdx.x - offs[ti]) * 256 + threadIdx.x;
  if (k >= d.p) return;
  double s = 0.0;
  for (int rc = 0; rc < d.nrowchunks; ++rc) s += d.colpart[(int64_t)rc * d.p + k];
  d.colmean[k] = s / (double)((int64_t)d.nx + d.ny);
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per padded pooled row: write W[pos][0..p_pad), nrm[pos]; flag NaN/Inf.
__global__ void __launch_bounds__(256) k_stage(const TestDesc* __restrict__ descs,
                                               const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  const int lane = threadIdx.x & 63;
  const int64_t pos = local * 4 + (threadIdx.x >> 6);
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
  if (d.prec == PREC_F64) {
    double* W = (double*)d.W + pos * d.p_pad;
    for (int k = lane; k < d.p_pad; k += 64) {
      double v = 0.0;
      if (t >= 0 && k < d.p) {
        v = load_in_f64(d, t, k);
        bad |= !isfinite(v);
      }
      W[k] = v;
      nrm += v * v;
    }
    nrm = wave_sum(nrm);
    if (lane == 0) ((double*)d.nrm)[pos] = nrm;
  } else {
    const bool bf = d.prec == PREC_BF16R;
    for (int k = lane; k < d.p_pad; k += 64) {
      float v = 0.0f;
      if (t >= 0 && k < d.p) {
        const float x = load_in_f32(d, t, k);
        bad |= !isfinite(x);
        v = (float)((double)x - d.colmean[k]);
      }
      if (bf) {
        const uint16_t h = f32_to_bf16_rn(v);
        ((uint16_t*)d.W)[pos * d.p_pad + k] = h;
        const float r = bf16_to_f32(h);
        nrm += (double)r * (double)r;
      } else {
        ((float*)d.W)[pos * d.p_pad + k] = v;
        nrm += (double)v * (double)v;
      }
    }
    nrm = wave_sum(nrm);
    if (lane == 0) ((float*)d.nrm)[pos] = (float)nrm;
  }
  if (bad) atomicOr(&d.flags[0], 1);
}

// Clear the per-test flag words (a kernel rather than a memset so that the
// launch sequence can be captured into a graph).  With a prefix table, only
// tests that own workgroups in it are cleared.
__global__ void k_clear_flags(const TestDesc* __restrict__ descs, const int64_t* __restrict__ offs,
                              int ntests) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntests && (offs == nullptr || offs[t + 1] > offs[t])) {
    descs[t].flags[0] = 0;
    descs[t].flags[1] = 0;
    descs[t].flags[2] = 0;
  }
}

void launch_clear_flags(hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  hipLaunchKernelGGL(k_clear_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, offs, n);
}
void launch_colpart(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_colpart, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}
void launch_colmean(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_colmean, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}
void launch_stage(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_stage, dim3((unsigned)blocks), dim3(256), 0, st, d, offs, n);
}

}  // namespace et
