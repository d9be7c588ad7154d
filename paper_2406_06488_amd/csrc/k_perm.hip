// Resampling stage.
//
// After double centring, every resampled statistic is +-(1/nx + 1/ny)^2 times
// z^T Dc z, where z is the split's 0/1 membership vector (see k_center.hip).
// For a batch of splits Z (n x P, columns = splits) the quantities needed are
// the diagonal of Z^T Dc Z: U = Dc Z is a dense contraction over pooled items,
// and q_c = sum_a Z[a,c] U[a,c] folds the row weights back in.  One workgroup
// takes one row tile i, a range of column tiles j >= i (only stored tiles are
// read: XX upper, XY, YY upper -- never D_YX) and NP = 256 split columns, and
// writes its FP64 partial of q for those columns.
//
// FP32 / BF16 forms: Dc is held as S bf16 planes whose sum is the FP32 value
// (S = 3 exact); membership bits expand to exact 0/1 bf16, so the products on
// v_mfma_f32_32x32x16_bf16 are exact and only FP32 accumulation order differs
// from an FP32 evaluation.  Partials over a row tile are reduced in FP64.
// FP64 form: the same quadratic form on the FP64 vector ALU.
#include "common.h"

namespace et {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t two_bits_bf16(uint32_t b) {
  // bit 0 -> low bf16 (1.0 = 0x3F80), bit 1 -> high bf16
  return ((b & 1u) * 0x3F80u) | (((b >> 1) & 1u) * 0x3F800000u);
}

__device__ inline uint4 expand_byte(uint32_t byte) {
  return make_uint4(two_bits_bf16(byte), two_bits_bf16(byte >> 2), two_bits_bf16(byte >> 4),
                    two_bits_bf16(byte >> 6));
}

// Workgroup: 4 waves; wave w owns rows 32w..32w+31 of the row tile and all NP
// split columns (8 blocks of 32) -> 8 accumulators of 32 x 32.
template <int S>
__global__ void __launch_bounds__(256) k_perm_mfma(const TestDesc* __restrict__ descs,
                                                   const int64_t* __restrict__ offs, int ntests,
                                                   const int32_t* __restrict__ pcr) {
  __shared__ uint4 Bl[8 * 8 * 64];  // B fragments of one column tile: [ks][nb][lane]
  __shared__ double red[4][NP];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc& d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  // split-column chunks of this launch: [pc0, pc0 + pcn) (all of them without a range table)
  const int pc0 = pcr ? pcr[2 * ti] : 0;
  const int pcn = pcr ? pcr[2 * ti + 1] : (int)(d.B_pad / NP);
  const int rk = (int)(local / pcn), pc = pc0 + (int)(local % pcn);
  int i, j0, j1;
  rowk_coords(d, rk, &i, &j0, &j1);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, lr = lane & 31;
  const int64_t colbase = (int64_t)pc * NP;
  f32x16 acc[8];
  for (int nb = 0; nb < 8; ++nb)
    for (int e = 0; e < 16; ++e) acc[nb][e] = 0.0f;
  const uint16_t* planes = (const uint16_t*)d.planes;
  const uint32_t* Z = d.Z;

  for (int j = j0; j < j1; ++j) {
    const int t = tile_index(i, j, d.nt);
    __syncthreads();
    {
      // thread tid expands split column colbase + tid for the 128 items of tile j
      uint32_t wq[TILE_WORDS];
      for (int q = 0; q < TILE_WORDS; ++q)
        wq[q] = Z[(int64_t)(j * TILE_WORDS + q) * d.B_pad + colbase + tid];
      const int nb = tid >> 5, pl = tid & 31;
      for (int ks = 0; ks < 8; ++ks)
        for (int hh = 0; hh < 2; ++hh) {
          const uint32_t byte = (wq[ks >> 1] >> ((ks & 1) * 16 + hh * 8)) & 0xFFu;
          Bl[(ks * 8 + nb) * 64 + pl + 32 * hh] = expand_byte(byte);
        }
    }
    __syncthreads();
    const uint16_t* At = planes + (int64_t)t * S * TILE * TILE + ((int64_t)(w * 8) * 64 + lane) * 8;
#pragma unroll 2
    for (int ks = 0; ks < 8; ++ks) {
      bf16x8 a[S];
#pragma unroll
      for (int s = 0; s < S; ++s) a[s] = *(const bf16x8*)(At + s * TILE * TILE + ks * 512);
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) {
        const uint4 bu = Bl[(ks * 8 + nb) * 64 + lane];
        const bf16x8 b = __builtin_bit_cast(bf16x8, bu);
#pragma unroll
        for (int s = 0; s < S; ++s)
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], b, acc[nb], 0, 0, 0);
      }
    }
  }
  // q_c partial: sum over this wave's rows a of z_c[a] * U[a, c]
  for (int nb = 0; nb < 8; ++nb) {
    const int64_t col = colbase + nb * 32 + lr;
    const uint32_t wz = Z[(int64_t)(i * TILE_WORDS + w) * d.B_pad + col];
    double q = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int bit = 8 * (e >> 2) + 4 * h + (e & 3);
      if ((wz >> bit) & 1u) q += (double)acc[nb][e];
    }
    q += __shfl_xor(q, 32, 64);
    if (h == 0) red[w][nb * 32 + lr] = q;
  }
  __syncthreads();
  const double s = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  d.part[(int64_t)rk * d.B_pad + colbase + tid] = s;
}

// FP64: thread = split column; rows of the centred tile are staged 32 at a time.
__global__ void __launch_bounds__(256) k_perm_f64(const TestDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ offs, int ntests,
                                                  const int32_t* __restrict__ pcr) {
  __shared__ double Ts[32 * TILE];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc& d = descs[ti];
  const int64_t local = blockIdx.x - offs[ti];
  // split-column chunks of this launch: [pc0, pc0 + pcn) (all of them without a range table)
  const int pc0 = pcr ? pcr[2 * ti] : 0;
  const int pcn = pcr ? pcr[2 * ti + 1] : (int)(d.B_pad / NP);
  const int rk = (int)(local / pcn), pc = pc0 + (int)(local % pcn);
  int i, j0, j1;
  rowk_coords(d, rk, &i, &j0, &j1);
  const int tid = threadIdx.x;
  const int64_t col = (int64_t)pc * NP + tid;
  const uint32_t* Z = d.Z;
  uint32_t zi[TILE_WORDS];
  for (int q = 0; q < TILE_WORDS; ++q) zi[q] = Z[(int64_t)(i * TILE_WORDS + q) * d.B_pad + col];
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) {
    uint32_t zj[TILE_WORDS];
    for (int q = 0; q < TILE_WORDS; ++q) zj[q] = Z[(int64_t)(j * TILE_WORDS + q) * d.B_pad + col];
    const double* Tt = (const double*)d.planes + (int64_t)tile_index(i, j, d.nt) * TILE * TILE;
    for (int rc = 0; rc < TILE_WORDS; ++rc) {
      __syncthreads();
      for (int e = tid; e < 32 * TILE; e += 256) Ts[e] = Tt[(int64_t)rc * 32 * TILE + e];
      __syncthreads();
      for (int rr = 0; rr < 32; ++rr) {
        double u = 0.0;
        for (int q = 0; q < TILE_WORDS; ++q) {
          const uint32_t wq = zj[q];
#pragma unroll 8
          for (int b = 0; b < 32; ++b)
            u = fma(Ts[rr * TILE + q * 32 + b], (double)((wq >> b) & 1u), u);
        }
        if ((zi[rc] >> rr) & 1u) acc += u;
      }
    }
  }
  d.part[(int64_t)rk * d.B_pad + col] = acc;
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
