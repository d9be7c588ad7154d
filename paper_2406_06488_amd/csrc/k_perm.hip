// Resampling stage.
//
// After double centring, every resampled statistic is +-(1/nx + 1/ny)^2 times
// z^T Dc z, where z is the split's 0/1 membership vector (see k_center.hip).
// For a batch of splits Z (n x P, columns = splits) the quantities needed are
// the diagonal of Z^T Dc Z: U = Dc Z is a dense contraction over pooled items,
// and q_c = sum_a Z[a,c] U[a,c] folds the row weights back in.  Only stored
// tiles are read (XX upper, XY, YY upper -- never D_YX); the halved diagonal
// tiles make z^T Dc z = 2 * sum over stored tiles (i <= j) of z_i^T T_ij z_j.
//
// Work unit: (row tile i, column tiles [j0, j1), split-column chunks [cb, ce)),
// chunk = NP = 256 splits.  FP32 / BF16 forms: wave w owns rows 32w..32w+31 of
// the row tile; the A fragments of its rows of tile (i, j) -- S bf16 planes whose
// sum is the centred FP32 value (S = 3 exact) -- are loaded once into registers
// and reused for every chunk; membership bits expand in registers to exact 0/1
// bf16 B fragments, so the products on v_mfma_f32_32x32x16_bf16 are exact.  Each
// (tile, chunk) product is folded into per-wave FP64 column sums in LDS; the
// four waves are added in a fixed order at the end.  FP64 form: the same
// quadratic form on the FP64 vector ALU, one thread per split.
#include "common.h"

namespace et {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t two_bits_bf16(uint32_t b) {
  // bit 0 -> low bf16 (1.0 = 0x3F80), bit 1 -> high bf16
  return ((b & 1u) * 0x3F80u) | (((b >> 1) & 1u) * 0x3F800000u);
}

__device__ inline bf16x8 expand_byte(uint32_t byte) {
  const uint4 u = make_uint4(two_bits_bf16(byte), two_bits_bf16(byte >> 2),
                             two_bits_bf16(byte >> 4), two_bits_bf16(byte >> 6));
  return __builtin_bit_cast(bf16x8, u);
}

struct PermUnit {
  int i, j0, j1, rk, cb, ce;
};

__device__ inline PermUnit perm_unit(const TestDesc& d, int ti, int64_t local,
                                     const int32_t* __restrict__ pcr) {
  // split-column chunks of this launch: [pc0, pc0 + pcn) (all of them without a range table)
  const int pc0 = pcr ? pcr[2 * ti] : 0;
  const int pcn = pcr ? pcr[2 * ti + 1] : (int)(d.B_pad / NP);
  const int ncr = (pcn + d.cc - 1) / d.cc;
  PermUnit u;
  u.rk = (int)(local / ncr);
  const int cr = (int)(local % ncr);
  u.cb = pc0 + cr * d.cc;
  u.ce = min(pc0 + pcn, u.cb + d.cc);
  rowk_coords(d, u.rk, &u.i, &u.j0, &u.j1);
  return u;
}

template <int S>
__global__ void __launch_bounds__(256) k_perm_mfma(const TestDesc* __restrict__ descs,
                                                   const int64_t* __restrict__ offs, int ntests,
                                                   const int32_t* __restrict__ pcr) {
  __shared__ double qs[4][MAX_CC][NP];  // per-wave FP64 column sums
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc& d = descs[ti];
  const PermUnit u = perm_unit(d, ti, blockIdx.x - offs[ti], pcr);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, lr = lane & 31;
  const int ncc = u.ce - u.cb;
  for (int e = lane; e < ncc * NP; e += 64) qs[w][e / NP][e % NP] = 0.0;
  const uint16_t* planes = (const uint16_t*)d.planes;
  const uint32_t* Z = d.Z;
  const int64_t BP = d.B_pad;

  for (int j = u.j0; j < u.j1; ++j) {
    const int t = tile_index(u.i, j, d.nt);
    bf16x8 a[8][S];
    const uint16_t* At = planes + (int64_t)t * S * TILE * TILE + ((int64_t)(w * 8) * 64 + lane) * 8;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
      for (int s = 0; s < S; ++s) a[ks][s] = *(const bf16x8*)(At + s * TILE * TILE + ks * 512);
    for (int c = u.cb; c < u.ce; ++c) {
      // membership words of column tile j (4 words = 128 items) for split c*NP + nb*32 + lr
      const uint32_t* Zc = Z + (int64_t)(j * TILE_WORDS) * BP + (int64_t)c * NP + lr;
      uint32_t zw[8][TILE_WORDS];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
#pragma unroll
        for (int q = 0; q < TILE_WORDS; ++q) zw[nb][q] = Zc[(int64_t)q * BP + nb * 32];
      // row bits of this wave's 32 rows of tile i
      uint32_t zr[8];
      const uint32_t* Zr = Z + (int64_t)(u.i * TILE_WORDS + w) * BP + (int64_t)c * NP + lr;
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) zr[nb] = Zr[nb * 32];
      f32x16 acc[8];
#pragma unroll
      for (int nb = 0; nb < 8; ++nb)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[nb][e] = 0.0f;
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
          const bf16x8 b = expand_byte((zw[nb][ks >> 1] >> ((ks & 1) * 16 + h * 8)) & 0xFFu);
#pragma unroll
          for (int s = 0; s < S; ++s)
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks][s], b, acc[nb], 0, 0, 0);
        }
      // fold the row weights: sum over this wave's rows a of z_c[a] * U[a, c]
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        double q = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int bit = 8 * (e >> 2) + 4 * h + (e & 3);
          if ((zr[nb] >> bit) & 1u) q += (double)acc[nb][e];
        }
        q += __shfl_xor(q, 32, 64);
        if (h == 0) qs[w][c - u.cb][nb * 32 + lr] += q;
      }
    }
  }
  __syncthreads();
  for (int c = 0; c < ncc; ++c) {
    const double s = ((qs[0][c][tid] + qs[1][c][tid]) + qs[2][c][tid]) + qs[3][c][tid];
    d.part[(int64_t)u.rk * BP + (int64_t)(u.cb + c) * NP + tid] = s;
  }
}

// FP64: thread = split column; rows of the centred tile are staged 32 at a time.
__global__ void __launch_bounds__(256) k_perm_f64(const TestDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ offs, int ntests,
                                                  const int32_t* __restrict__ pcr) {
  __shared__ double Ts[32 * TILE];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc& d = descs[ti];
  const PermUnit u = perm_unit(d, ti, blockIdx.x - offs[ti], pcr);
  const int tid = threadIdx.x;
  const uint32_t* Z = d.Z;
  for (int c = u.cb; c < u.ce; ++c) {
    const int64_t col = (int64_t)c * NP + tid;
    uint32_t zi[TILE_WORDS];
    for (int q = 0; q < TILE_WORDS; ++q) zi[q] = Z[(int64_t)(u.i * TILE_WORDS + q) * d.B_pad + col];
    double acc = 0.0;
    for (int j = u.j0; j < u.j1; ++j) {
      uint32_t zj[TILE_WORDS];
      for (int q = 0; q < TILE_WORDS; ++q) zj[q] = Z[(int64_t)(j * TILE_WORDS + q) * d.B_pad + col];
      const double* Tt = (const double*)d.planes + (int64_t)tile_index(u.i, j, d.nt) * TILE * TILE;
      for (int rc = 0; rc < TILE_WORDS; ++rc) {
        __syncthreads();
        for (int e = tid; e < 32 * TILE; e += 256) Ts[e] = Tt[(int64_t)rc * 32 * TILE + e];
        __syncthreads();
        for (int rr = 0; rr < 32; ++rr) {
          double v = 0.0;
          for (int q = 0; q < TILE_WORDS; ++q) {
            const uint32_t wq = zj[q];
#pragma unroll 8
            for (int b = 0; b < 32; ++b)
              v = fma(Ts[rr * TILE + q * 32 + b], (double)((wq >> b) & 1u), v);
          }
          if ((zi[rc] >> rr) & 1u) acc += v;
        }
      }
    }
    d.part[(int64_t)u.rk * d.B_pad + col] = acc;
  }
}

void launch_perm(int variant, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int ntests, const int32_t* pcr) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  switch (variant) {
    case 0: hipLaunchKernelGGL(k_perm_f64, g, b, 0, st, d, offs, ntests, pcr); break;
    case 1: hipLaunchKernelGGL(k_perm_mfma<1>, g, b, 0, st, d, offs, ntests, pcr); break;
    case 2: hipLaunchKernelGGL(k_perm_mfma<2>, g, b, 0, st, d, offs, ntests, pcr); break;
    default: hipLaunchKernelGGL(k_perm_mfma<3>, g, b, 0, st, d, offs, ntests, pcr); break;
  }
}

}  // namespace et
