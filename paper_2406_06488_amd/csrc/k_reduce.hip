// Pooled row sums and the observed statistic.
//
// For pooled position a in row tile i, the same-sample part of its row sum
// gathers row sums of tiles (i, j >= i) and column sums of tiles (j < i, i)
// inside its own block (XX or YY); the cross-sample part gathers the XY tiles
// (row sums for an X position, column sums for a Y position).  Summing the
// parts over positions gives S_XX, S_YY and S_XY, the three block sums of
// eq. (1) / eq. (2), accumulated with Neumaier compensation in FP64.
#include "common.h"

namespace et {

// Thread q < npad: same-sample part of position q; q >= npad: cross-sample part of
// position q - npad.  One wave per workgroup so that the short grid spreads over the CUs.
__global__ void __launch_bounds__(64) k_rowsum(const TestDesc* __restrict__ descs,
                                               const int64_t* __restrict__ offs, int ntests) {
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int64_t npad = (int64_t)d.nt * TILE;
  const int64_t q = (blockIdx.x - offs[ti]) * 64 + threadIdx.x;
  if (q >= 2 * npad) return;
  const bool cross = q >= npad;
  const int64_t pos = cross ? q - npad : q;
  const int i = (int)(pos / TILE), r = (int)(pos % TILE);
  const double* ts = d.tsum;
  const bool isx = i < d.tx;
  double s = 0.0;
  // row sums of tile (i, j); column sums (two row halves) of tile (j, i)
  auto rowsum = [&](int j) { return ts[(int64_t)tile_index(i, j, d.nt) * TSUM_STRIDE + r]; };
  auto colsum = [&](int j) {
    const double* t = ts + (int64_t)tile_index(j, i, d.nt) * TSUM_STRIDE;
    return t[TILE + r] + t[2 * TILE + r];
  };
  // unrolled so that several tile sums are in flight; the additions stay in order of j
  if (!cross) {
    const int b0 = isx ? 0 : d.tx, b1 = isx ? d.tx : d.nt;  // own block's tile range
#pragma unroll 8
    for (int j = b0; j < i; ++j) s += colsum(j);
#pragma unroll 8
    for (int j = i; j < b1; ++j) s += rowsum(j);
  } else if (isx) {
#pragma unroll 8
    for (int j = d.tx; j < d.nt; ++j) s += rowsum(j);
  } else {
#pragma unroll 8
    for (int j = 0; j < d.tx; ++j) s += colsum(j);
  }
  d.rsum[pos * 2 + (cross ? 1 : 0)] = s;
}

constexpr int OBS_BATCH = 8;

struct Neu {
  double s, c;
  __device__ void add(double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

// One workgroup per test: S_XX, S_YY, S_XY and the observed statistic.
__global__ void __launch_bounds__(256) k_observed(const TestDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ sel, int ntests) {
  __shared__ double red[3][256][2];
  if (sel && sel[blockIdx.x + 1] == sel[blockIdx.x]) return;
  const TestDesc d = descs[blockIdx.x];
  const int tid = threadIdx.x;
  Neu sxx{0, 0}, syy{0, 0}, sxy{0, 0};
  const int64_t xend = (int64_t)d.tx * TILE, npad = (int64_t)d.nt * TILE;
  // The loads of OBS_BATCH positions are issued together before any of them is added (the
  // row sums were just written by other XCDs, so each load waits on a far cache); the
  // additions keep the order pos = tid, tid + 256, ... .
  for (int64_t base = tid; base < npad; base += 256 * OBS_BATCH) {
    double a[OBS_BATCH], b[OBS_BATCH];
#pragma unroll
    for (int u = 0; u < OBS_BATCH; ++u) {
      const int64_t pos = base + 256 * u;
      a[u] = pos < npad ? d.rsum[pos * 2] : 0.0;
      b[u] = pos < xend ? d.rsum[pos * 2 + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < OBS_BATCH; ++u) {
      const int64_t pos = base + 256 * u;
      if (pos < xend) {
        sxx.add(a[u]);
        sxy.add(b[u]);
      } else if (pos < npad) {
        syy.add(a[u]);
      }
    }
  }
  red[0][tid][0] = sxx.s; red[0][tid][1] = sxx.c;
  red[1][tid][0] = syy.s; red[1][tid][1] = syy.c;
  red[2][tid][0] = sxy.s; red[2][tid][1] = sxy.c;
  // pairwise combination of the compensated partials (fixed tree: reproducible)
  for (int st = 128; st > 0; st >>= 1) {
    __syncthreads();
    if (tid < st)
      for (int a = 0; a < 3; ++a) {
        Neu u{red[a][tid][0], red[a][tid][1] + red[a][tid + st][1]};
        u.add(red[a][tid + st][0]);
        red[a][tid][0] = u.s;
        red[a][tid][1] = u.c;
      }
  }
  __syncthreads();
  if (tid < 3) d.obs[tid] = red[tid][0][0] + red[tid][0][1];
  __syncthreads();
  if (tid == 0) {
    const double nx = d.nx, ny = d.ny;
    const double txx = d.obs[0] / (nx * nx), tyy = d.obs[1] / (ny * ny);
    const double txy = 2.0 * d.obs[2] / (nx * ny);
    d.obs[3] = d.kind == KIND_ED ? (txy - txx) - tyy : (txx + tyy) - txy;
    d.obs[4] = d.obs[0] + d.obs[1] + 2.0 * d.obs[2];  // R = sum of all pooled row sums
  }
  // Scale of the fp16 planes of the FP32 / BF16 forms: a centred entry
  // D - c_a - c_b + c0 (all of them within [0, max D] for distances and kernel values)
  // is at most 4 max|D| in size; scaling by 2^e with 4 max|D| 2^e <= 2^14 keeps every
  // plane value inside the fp16 range.
  __shared__ float mx[256];
  float m = 0.0f;
  if (d.prec != PREC_F64) {
    const int nmax = d.ntiles * TMAX_PER_TILE;
    for (int base = tid; base < nmax; base += 256 * OBS_BATCH) {
      float v[OBS_BATCH];
#pragma unroll
      for (int u = 0; u < OBS_BATCH; ++u) v[u] = base + 256 * u < nmax ? d.tmax[base + 256 * u] : 0.0f;
#pragma unroll
      for (int u = 0; u < OBS_BATCH; ++u) m = fmaxf(m, v[u]);
    }
  }
  mx[tid] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) mx[tid] = fmaxf(mx[tid], mx[tid + s]);
    __syncthreads();
  }
  if (tid == 0) {
    const double bound = 4.0 * (double)mx[0];
    int e = 0;
    if (bound > 0.0) e = 14 - (int)ceil(log2(bound));
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
    d.obs[5] = ldexp(1.0, e);
  }
}

void launch_rowsum(int64_t blocks, hipStream_t st, const TestDesc* d, const int64_t* offs, int n) {
  if (blocks > 0) hipLaunchKernelGGL(k_rowsum, dim3((unsigned)blocks), dim3(64), 0, st, d, offs, n);
}
void launch_observed(hipStream_t st, const TestDesc* d, const int64_t* sel, int n) {
  hipLaunchKernelGGL(k_observed, dim3((unsigned)n), dim3(256), 0, st, d, sel, n);
}

}  // namespace et
