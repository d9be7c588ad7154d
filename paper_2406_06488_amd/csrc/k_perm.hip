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
// chunk = NP = 256 splits.  FP32 / BF16 forms: the centred tiles are held as two planes
// (see k_center.hip).  FP32 form: fp16 hi and lo (value = hi + lo 2^-11); membership bits
// expand to exact fp16 B fragments worth 1 (for hi) and 2^-11 (for lo), both multiplied on
// v_mfma_f32_32x32x16_f16.  BF16-refined form: fp16 hi as above and an e4m3 lo plane
// (value = hi + lo 2^-5), whose bits expand to fp8 bytes worth 2^-5 for
// v_mfma_scale_f32_32x32x64_f8f6f4 (unit block scales), which takes 64 columns per
// instruction at about 1.6x the fp16 rate.  Every product is exact, so only the FP32
// accumulation order differs from an exact evaluation; partial sums per row range are
// reduced in FP64.  FP64 form: the same quadratic form on the FP64 vector ALU, one thread
// per split.
#include "common.h"

namespace et {

typedef float f32x16 __attribute__((ext_vector_type(16)));


typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// 8 membership bits -> 8 fp16 values 0.0 / 1.0 (element k = bit k).  m = byte * 0x8001
// holds bit k at positions k and k + 15, so dword q's two bits 2q and 2q+1 sit at positions
// 2q and 2q + 16; masking them in place and multiplying by 0x3C00 >> 2q (an integer, as
// 0x3C00 = 15 * 2^10) puts fp16 1.0 at bits 0 and 16.
__device__ inline uint4 expand_byte(uint32_t byte) {
  const uint32_t m = byte * 0x8001u;
  return make_uint4((m & 0x10001u) * 0x3C00u, (m & 0x40004u) * 0x0F00u,
                    (m & 0x100010u) * 0x03C0u, (m & 0x400040u) * 0x00F0u);
}
// The same bits worth 2^-11 (fp16 0x1000) for the low plane: 0x3C00 & 0x1000 = 0x1000.
__device__ inline uint4 low_weights(uint4 u) {
  return make_uint4(u.x & 0x10001000u, u.y & 0x10001000u, u.z & 0x10001000u, u.w & 0x10001000u);
}

// 32 membership bits (bit j = column j of a 64-column step's lane group) -> 32 fp8 E4M3
// bytes worth 2^-5 (code 0x10) or 0.  Nibble q, placed at bits 4..7, times 0x204081 puts
// bit i of the nibble at bit 4 + 8 i (the four shifted copies do not collide there).
__device__ inline i32x8 expand_word_e4m3(uint32_t w) {
  i32x8 o;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const uint32_t nib16 = q == 0 ? (w << 4) & 0xF0u : (w >> (4 * q - 4)) & 0xF0u;
    o[q] = (int)((nib16 * 0x204081u) & 0x10101010u);
  }
  return o;
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

// Workgroup: 8 waves over two chunks of 256 split columns; wave w owns columns
// (w & 3) * 64 .. + 63 of chunk w >> 2 and all 128 rows of the row tile (4 row blocks x 2
// column blocks of 32 x 32 accumulators).  The A tile (i, j) -- S fp16 planes in
// fragment order -- and the membership words of column tile j stream straight into one
// of two LDS buffers (global_load_lds) while the other buffer is multiplied.  Each wave
// folds the row weights of its own columns at the end: no cross-wave reduction.

__device__ inline void load_to_lds16(const void* g, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds_wave_base, 16,
                                   0, 0);
}

template <int S>
__global__ void __launch_bounds__(PERM_THREADS) k_perm_mfma(const TestDesc* __restrict__ descs,
                                                            const int64_t* __restrict__ offs,
                                                            int ntests,
                                                            const int32_t* __restrict__ pcr) {
  constexpr int FR = TILE * TILE / 8;         // 16-byte fragments per plane (2048)
  constexpr int ZW = TILE_WORDS * 2 * NP / 4;  // 16-byte groups of membership words (512)
  constexpr int PU = S == 3 ? FR + FR / 2 : S * FR;  // 16-byte slots of one tile's planes
  constexpr int BUF = PU + ZW;                // 16-byte slots per buffer
  __shared__ uint4 lds[2 * BUF];
  const int64_t bid = xcd_grouped(blockIdx.x, gridDim.x);
  const int ti = find_test(offs, ntests, bid);
  const TestDesc d = descs[ti];
  const PermUnit u = perm_unit(d, ti, bid - offs[ti], pcr);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, lr = lane & 31;
  const int64_t BP = d.B_pad;
  const int nch = u.ce - u.cb;  // 1 or 2
  const int cw = w >> 2;        // this wave's chunk
  const bool active = cw < nch;
  const uint4* planes = (const uint4*)d.planes;
  const uint32_t* Z = d.Z;
  const int lcol = cw * NP + (w & 3) * 64 + lr;  // column within the workgroup's 512 (nb = 0)

  // Queue the A tile and membership words of column tile j into buffer `buf`.
  auto issue = [&](int j, int buf) {
    uint4* dst = lds + buf * BUF;
    const uint4* src = planes + (int64_t)tile_index(u.i, j, d.nt) * PU;
#pragma unroll
    for (int r = 0; r < PU / PERM_THREADS; ++r) {
      const int q = tid + PERM_THREADS * r;
      load_to_lds16(src + q, dst + (q - lane));
    }
    // words (j*4 + q) of the 512 columns: 128 lanes x 16 bytes per word row q
    const int q = tid >> 7, part = tid & 127;
    if (part * 4 < nch * NP) {
      const uint32_t* zsrc =
          Z + (int64_t)(j * TILE_WORDS + q) * BP + (int64_t)u.cb * NP + part * 4;
      load_to_lds16(zsrc, dst + PU + (tid - lane));
    }
  };

  // row weights for the final fold, fetched now so their latency hides behind the tiles
  uint32_t wzf[2][4];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
      wzf[nb][mb] = active ? Z[(int64_t)(u.i * TILE_WORDS + mb) * BP + (int64_t)u.cb * NP + lcol +
                               nb * 32]
                           : 0u;
  f32x16 acc[4][2];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mb][nb][e] = 0.0f;

  issue(u.j0, 0);
  for (int j = u.j0; j < u.j1; ++j) {
    const int buf = (j - u.j0) & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads into `buf` have landed
    __syncthreads();                // everyone's have, and `buf ^ 1` is free again
    if (j + 1 < u.j1) issue(j + 1, buf ^ 1);
    const uint4* A = lds + buf * BUF;
    const uint32_t* zl = (const uint32_t*)(A + PU);  // [q][512 columns]
    if (active) {
      uint32_t zw[2][TILE_WORDS];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int q = 0; q < TILE_WORDS; ++q) zw[nb][q] = zl[q * 2 * NP + lcol + nb * 32];
      // A fragments of step ks + 1 are read from LDS while step ks is multiplied.  NH fp16
      // planes; with the e4m3 low plane (S == 3) its fragments cover 64 columns (4 steps)
      // and are read at the first step of each 64.
      constexpr int NH = S == 3 ? 1 : S;
      const uint4* Alo = A + FR;  // e4m3 plane: [fragment (mb, kb)][half][lane]
      f16x8 a[4][NH], an[4][NH];
      i32x8 al[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int s = 0; s < NH; ++s)
          a[mb][s] = __builtin_bit_cast(f16x8, A[s * FR + (mb * 8) * 64 + lane]);
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        // this step's fragments (read one step earlier) have landed; waiting here, before
        // the next reads are issued, keeps at most 12 LDS reads in flight
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unconstrained
        __builtin_amdgcn_sched_barrier(0);
        if (S == 3 && (ks & 3) == 0) {
          const int kb = ks >> 2;
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            const uint4 p0 = Alo[((mb * 2 + kb) * 2 + 0) * 64 + lane];
            const uint4 p1 = Alo[((mb * 2 + kb) * 2 + 1) * 64 + lane];
            al[mb] = i32x8{(int)p0.x, (int)p0.y, (int)p0.z, (int)p0.w,
                           (int)p1.x, (int)p1.y, (int)p1.z, (int)p1.w};
          }
        }
        if (ks + 1 < 8) {
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int s = 0; s < NH; ++s)
              an[mb][s] = __builtin_bit_cast(f16x8, A[s * FR + (mb * 8 + ks + 1) * 64 + lane]);
        }
        // keep those reads ahead of this step's products (the scheduler would otherwise
        // sink them and wait on them before the first product)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const uint4 bu = expand_byte((zw[nb][ks >> 1] >> ((ks & 1) * 16 + h * 8)) & 0xFFu);
          const f16x8 b1 = __builtin_bit_cast(f16x8, bu);
          const f16x8 b2 = __builtin_bit_cast(f16x8, low_weights(bu));
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[mb][0], b1, acc[mb][nb], 0, 0, 0);
            if (S == 2)
              acc[mb][nb] =
                  __builtin_amdgcn_mfma_f32_32x32x16_f16(a[mb][NH - 1], b2, acc[mb][nb], 0, 0, 0);
          }
        }
        if (S == 3 && (ks & 3) == 0) {
          // columns 64 kb + 32 h + j of lane group h are bit j of membership word 2 kb + h
          const int kb = ks >> 2;
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            const i32x8 b8 = expand_word_e4m3(h ? zw[nb][2 * kb + 1] : zw[nb][2 * kb]);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
              acc[mb][nb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                  al[mb], b8, acc[mb][nb], 0, 0, 0, 127, 0, 127);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int s = 0; s < NH; ++s) a[mb][s] = an[mb][s];
      }
    }
  }
  if (!active) return;
  // fold the row weights: q_c = sum over the tile's rows a of z_c[a] * U[a, c]
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int64_t col = (int64_t)u.cb * NP + lcol + nb * 32;
    double q = 0.0;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      // bit (8 (e / 4) + 4 h + e % 4) of the word weights element e; a sign-extended one-bit
      // field is an all-ones or all-zero mask, so a cleared bit adds +0.0 as before
      const uint32_t wz = wzf[nb][mb] >> (4 * h);
      float f = 0.0f;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)wz, 8 * (e >> 2) + (e & 3), 1);
        const float x = acc[mb][nb][e];  // a copy: a vector element has no address of its own
        f += __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) & m);
      }
      q += (double)f;
    }
    q += __shfl_xor(q, 32, 64);
    if (h == 0) d.part[(int64_t)u.rk * BP + col] = q;
  }
}

// FP64: thread = split column (a workgroup covers 256 columns of a chunk); each workgroup
// takes one 32-row strip of its row unit's centred tiles (the row units of an FP64 test are
// PC_STRIPS times as many as its row-unit walk gives: unit rks = row unit rks / PC_STRIPS,
// strip rks % PC_STRIPS), so that even a test of two tiles spreads over several CUs.
__global__ void __launch_bounds__(256) k_perm_f64(const TestDesc* __restrict__ descs,
                                                  const int64_t* __restrict__ offs, int ntests,
                                                  const int32_t* __restrict__ pcr) {
  __shared__ double Ts[PC_ROWS * TILE];
  const int ti = find_test(offs, ntests, blockIdx.x);
  const TestDesc d = descs[ti];
  const int pc0 = pcr ? pcr[2 * ti] : 0;
  const int pcn = pcr ? pcr[2 * ti + 1] : (int)(d.B_pad / NP);
  const int ncr = (pcn + d.cc - 1) / d.cc;
  const int64_t local = blockIdx.x - offs[ti];
  const int rks = (int)(local / ncr);
  const int cr = (int)(local % ncr);
  const int h = rks % PC_STRIPS;
  int i, j0, j1;
  rowk_coords(d, rks / PC_STRIPS, &i, &j0, &j1);
  const int cb = pc0 + cr * d.cc, ce = min(pc0 + pcn, cb + d.cc);
  const int tid = threadIdx.x;
  const uint32_t* Z = d.Z;
  constexpr int NLD = PC_ROWS * TILE / 2 / 256;  // 16-byte loads per thread per strip
  for (int c = cb; c < ce; ++c) {
    const int64_t col = (int64_t)c * NP + tid;
    const uint32_t zi = Z[(int64_t)(i * TILE_WORDS + h) * d.B_pad + col];
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
      uint32_t zj[TILE_WORDS];
#pragma unroll
      for (int q = 0; q < TILE_WORDS; ++q) zj[q] = Z[(int64_t)(j * TILE_WORDS + q) * d.B_pad + col];
      const double2* Tt = (const double2*)((const double*)d.planes +
                                           (int64_t)tile_index(i, j, d.nt) * TILE * TILE +
                                           (int64_t)h * PC_ROWS * TILE);
      double2 v[NLD];  // every load of the strip in flight before the first LDS store
#pragma unroll
      for (int k = 0; k < NLD; ++k) v[k] = Tt[tid + 256 * k];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NLD; ++k) ((double2*)Ts)[tid + 256 * k] = v[k];
      __syncthreads();
      for (int rr = 0; rr < PC_ROWS; ++rr) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < TILE_WORDS; ++q) {
          const uint32_t wq = zj[q];
#pragma unroll
          for (int b = 0; b < 32; ++b)
            a[b & 3] = fma(Ts[rr * TILE + q * 32 + b], (double)((wq >> b) & 1u), a[b & 3]);
        }
        if ((zi >> rr) & 1u) acc += (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
    d.part[(int64_t)rks * d.B_pad + col] = acc;
  }
}

void launch_perm(int variant, int64_t blocks, hipStream_t st, const TestDesc* d,
                 const int64_t* offs, int ntests, const int32_t* pcr) {
  if (blocks <= 0) return;
  const dim3 g((unsigned)blocks), b(256);
  switch (variant) {
    case 0: hipLaunchKernelGGL(k_perm_f64, g, b, 0, st, d, offs, ntests, pcr); break;
    case 2: hipLaunchKernelGGL(k_perm_mfma<2>, g, dim3(PERM_THREADS), 0, st, d, offs, ntests, pcr); break;
    case 3: hipLaunchKernelGGL(k_perm_mfma<3>, g, dim3(PERM_THREADS), 0, st, d, offs, ntests, pcr); break;
    default: break;
  }
}

}  // namespace et
