// Cross tests: cross-MMD (Alg. 6) and cross-ED (Alg. 7) of the paper's appendix.
//
// x is cut into x1 (its first floor(nx/2) rows) and x2, y into y1 and y2.  The block stage
// runs on the "x side" [x1; y1] against the "y side" [x2; y2] (the four cross blocks form
// that rectangle) and leaves, per tile and x-side row, the row's sums over the x2 columns
// and over the y2 columns.  Here, per x-side row a, with row means m2(a) over x2 and
// m3(a) over y2:
//   v(a) = m3(a) - m2(a) (ED)  or  m2(a) - m3(a) (MMD),
// so that U_x = mean of v over the x1 rows and U_y = mean of v over the y1 rows are the
// algorithms' differences of block means (a block mean is the mean of its row means);
//   U = U_x - U_y,  s_x = mean over x1 rows of (v - U_x)^2,  s_y likewise over y1 rows,
//   sigma = sqrt(s_x / |x1| + s_y / |y1|),  p = 1 - Phi(U / sigma) = erfc(z / sqrt 2) / 2.
// sigma = 0 gives z = +inf, -inf or 0 by the sign of U.  All sums are FP64 with
// compensation.
#include "common.h"

namespace et {

namespace {
struct Csum {  // compensated FP64 sum (Neumaier)
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};
}  // namespace

constexpr int CF_THREADS = 1024;

// Workgroup-wide sums of two values (every thread returns them).
__device__ inline void block_sum2(double& a, double& b, double (*red)[CF_THREADS / 64]) {
  for (int m = 32; m > 0; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int k = 0; k < CF_THREADS / 64; ++k) {
    a += red[0][k];
    b += red[1][k];
  }
}

__global__ void __launch_bounds__(CF_THREADS) k_cross_final(const TestDesc* __restrict__ descs) {
  __shared__ double red[2][CF_THREADS / 64];
  const TestDesc d = descs[0];
  const int64_t n_side = d.nx;  // x-side rows: x1 then y1
  const int64_t nx1 = d.cnx1, ny1 = d.cny1, nx2 = d.cnx2, ny2 = (int64_t)d.ny - d.cnx2;
  const bool ed = d.kind == KIND_ED;
  double* v = d.rsum;  // v(a) of every x-side row
  Csum sx, sy;
  for (int64_t a = threadIdx.x; a < n_side; a += CF_THREADS) {
    const int64_t i = a / TILE, r = a % TILE;
    Csum s2, s3;
    for (int jc = 0; jc < d.ty; ++jc) {
      const double* ts = d.tsum + (i * d.ty + jc) * TSUM_STRIDE;
      s2.add(ts[r]);
      s3.add(ts[TILE + r]);
    }
    const double m2 = s2.value() / (double)nx2, m3 = s3.value() / (double)ny2;
    const double val = ed ? m3 - m2 : m2 - m3;
    v[a] = val;
    if (a < nx1) sx.add(val);
    else sy.add(val);
  }
  double tx = sx.value(), ty = sy.value();
  block_sum2(tx, ty, red);
  const double ux = tx / (double)nx1, uy = ty / (double)ny1;
  Csum qx, qy;
  for (int64_t a = threadIdx.x; a < n_side; a += CF_THREADS) {
    const double dev = v[a] - (a < nx1 ? ux : uy);  // this thread wrote v[a] above
    if (a < nx1) qx.add(dev * dev);
    else qy.add(dev * dev);
  }
  double vx = qx.value(), vy = qy.value();
  block_sum2(vx, vy, red);
  if (threadIdx.x == 0) {
    const double u = ux - uy;
    const double sigma = sqrt((vx / (double)nx1) / (double)nx1 + (vy / (double)ny1) / (double)ny1);
    double z;
    if (sigma > 0.0) z = u / sigma;
    else z = u > 0.0 ? INFINITY : (u < 0.0 ? -INFINITY : 0.0);
    d.obs[0] = u;
    d.obs[1] = sigma;
    d.obs[2] = z;
    d.obs[3] = 0.5 * erfc(z * 0.70710678118654752440);
  }
}

void launch_cross_final(hipStream_t st, const TestDesc* d) {
  hipLaunchKernelGGL(k_cross_final, dim3(1), dim3(CF_THREADS), 0, st, d);
}

}  // namespace et
