// Shared definitions of the gfx950 kernels and the host runtime.
//
// Data layout in HBM for one test (n_pad = (tx + ty) * TILE):
//   W      staged operand rows: X rows, zero rows up to a TILE boundary, Y rows, zero
//          rows (column-mean centred for the FP32/BF16 forms).  FP64 operands row-major
//          [n_pad][p_pad]; 16-bit operands (BF16 values, or fp16 pairs hi/lo of the
//          scaled value) K-blocked [n_pad / T][p_pad / CK][T][32 halves] (blocked_index)
//   nrm    [n_pad]          squared row norms of the staged rows
//   D      [ntiles][T][T]   upper tiles (i <= j) of the pooled tile grid: XX upper
//                           tiles, every XY tile, YY upper tiles -- never a YX tile
//   tsum   [ntiles][2][T]   FP64 row / column sums of each stored tile
//   rsum   [n_pad][2]       pooled row sums: same-sample part, cross-sample part
//   planes [ntiles][S][T*T] double-centred tiles, scaled by a power of two and split
//                           into fp16 planes (hi, lo * 2^11) in MFMA A-fragment
//                           order (FP64 form: one FP64 row-major tile)
//   Z      [n_pad/32][B_pad] split membership bits, word w of column c holds items
//                           32w..32w+31; columns 0..B-1 drawn splits, column B the
//                           identity split, the rest zero
//   part   [n_rowk][B_pad]  FP64 partial quadratic forms per (row tile, column range)
//   pstat  [B_pad]          resampled statistics
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace et {

constexpr int TILE = 128;            // edge of a stored block tile
constexpr int TILE_WORDS = TILE / 32;
// Per stored tile: FP64 row sums [0, TILE), column sums of rows 0..63 [TILE, 2 TILE) and of
// rows 64..127 [2 TILE, 3 TILE); two tile-max slots (one per row half).
constexpr int TSUM_STRIDE = 3 * TILE;
constexpr int TMAX_PER_TILE = 2;
constexpr int NP = 256;              // split columns per resampling chunk
constexpr int MAX_CC = 8;            // chunks per resampling workgroup, at most
constexpr int COLSUM_ROWS = 32;      // pooled rows per partial column sum
constexpr int MEMBER_SPLITS = 16;    // split columns per split-stream workgroup
constexpr int MEMBER_SPLITS_WIDE = 32;  // the same for split streams larger than the chip
constexpr int FLAG_COUNT = 4;        // int32 index of the 64-bit (count, finished WGs) word
constexpr int FLAG_WORDS = 8;
constexpr int FLAG_XMAX = 6;         // FP32 form: bits of max |input| (a non-negative float)
constexpr int HSIC_NMAX = 4096;      // HSIC test: largest n (one sort and one kernel row in LDS)
constexpr int HSIC_RB = 8;           // HSIC test: rows of Kt per workgroup of the term pass
constexpr int PC_ROWS = 32;          // pre-computation test: tile rows per strip
constexpr int PC_STRIPS = TILE / PC_ROWS;
// Threads per workgroup of the kernels whose launch sizes the host checks.
constexpr int CM_GROUPS = 16;        // column-mean pass: 64-thread groups per workgroup
constexpr int MTHREADS = 256;        // split stream: wave 0 scans, waves 1..3 draw
constexpr int PERM_THREADS = 512;    // MFMA resampling: 8 waves
constexpr int PS_GROUPS = 16;        // split statistics: 64-thread groups per workgroup
// Largest pooled tile grid of one test (tx + ty tiles, nx and ny each padded to whole
// tiles): for nt <= 46340 the stored tile count nt (nt + 1) / 2 and every intermediate of
// the triangular tile index (i * nt) stay below 2^31.  That is 5.9 million pooled rows,
// whose blocks (~70 TB) no single GPU holds; requests beyond it are rejected as invalid.
constexpr int64_t MAX_TILE_GRID = 46340;

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16R = 2 };
// Operand format of the Gram (and of the staged rows it reads): FP64 rows (direct
// differences), fp16 pairs (hi, lo) of the scaled centred value (FP32-accurate products),
// or BF16 values.  The FP32 form uses fp16 pairs; the BF16-refined form uses BF16 operands
// from BF16_PAIR_MAX_P coordinates on and fp16 pairs below, where 8-bit coordinates move a
// distance by ~2^-9 / sqrt(p) of itself (beyond the form's 1e-3 statistic bound at p = 10)
// and the Gram is a negligible share of the test.
enum { GOP_F64 = 0, GOP_F16PAIR = 1, GOP_BF16 = 2 };
constexpr int BF16_PAIR_MAX_P = 64;
__host__ __device__ inline int gram_operands(int prec, int64_t p) {
  return prec == PREC_F64 ? GOP_F64
         : (prec == PREC_F32 || p < BF16_PAIR_MAX_P) ? GOP_F16PAIR : GOP_BF16;
}
// Gram workgroup shapes: one stored 128 x 128 tile per workgroup (four waves of 64 x 64),
// or one 2 x 2 block of stored tiles (a 256 x 256 super tile: four waves, one tile each).
enum { GSHAPE_TILE = 0, GSHAPE_SUPER = 1 };
// K-slice width of each Gram kernel: staged rows are padded to a multiple of it.
__host__ __device__ inline int gram_k_slice(int gop) {
  return gop == GOP_F64 ? 16 : (gop == GOP_F16PAIR ? 32 : 64);
}
// K-blocked layout of the 16-bit operands: every staged row is cut into chunks of 64
// bytes (BF16: 32 coordinates; fp16 pairs: 16 coordinates, their hi halves then their lo
// halves), and the chunks of one 128-row tile at one chunk position are contiguous (8 KB),
// so that a wave loads the chunks of 16 consecutive rows as one contiguous kilobyte.
constexpr int CHUNK_HALVES = 32;  // 16-bit values per row and chunk
__host__ __device__ inline int chunk_coords(int gop) { return gop == GOP_BF16 ? 32 : 16; }
// uint16 index of value c (0..31) of chunk `chunk` of staged row `row`
__host__ __device__ inline int64_t blocked_index(int64_t row, int64_t chunk, int c,
                                                 int64_t nchunks) {
  return (((row / TILE) * nchunks + chunk) * TILE + (row % TILE)) * CHUNK_HALVES + c;
}
// Bytes per staged operand element: FP64, one fp16 pair, one BF16 value.
__host__ __device__ inline int gram_operand_bytes(int gop) {
  return gop == GOP_F64 ? 8 : (gop == GOP_F16PAIR ? 4 : 2);
}
enum { KIND_ED = 0, KIND_MMD = 1 };

// Result written by the device (the public etest_result plus a status word).
struct DevResult {
  double statistic, threshold, p_value;
  int64_t count_ge, B, n_refined;
  int32_t status, pad;
};

// Plane formats of the centred tiles that the resampling stage multiplies (FP32 and
// BF16-refined forms; the FP64 form keeps FP64 tiles):
//  PLANES_F16_F16:  hi = fp16(v), lo = fp16((v - hi) 2^11); v to ~2^-22 of itself.
//  PLANES_F16_E4M3: hi = fp16(v), lo = e4m3((v - hi) 2^5) (fp8, OCP); v to ~2^-15.
constexpr int PLANES_F16_F16 = 2;
constexpr int PLANES_F16_E4M3 = 3;
__host__ __device__ inline int plane_bytes_per_entry(int pfmt) {
  return pfmt == PLANES_F16_E4M3 ? 3 : 4;
}

struct TestDesc {
  int32_t kind, prec, pfmt, refine;  // pfmt: plane format of the centred tiles (PLANES_*)
  int32_t gop, gshape;               // Gram operand format (GOP_*) and workgroup shape
                                     // (GSHAPE_*)
  int32_t nx, ny, p, p_pad;
  int32_t tx, ty, nt, ntiles;
  int32_t kc, n_rowk, nrowchunks, cc;  // cc: split-column chunks per resampling workgroup
  int64_t B, B_pad;
  uint64_t seed;
  double gamma;
  const void* X;
  const void* Y;
  double* colpart;
  double* colmean;
  void* W;
  void* nrm;
  void* D;
  double* tsum;
  float* tmax;       // [ntiles][2] largest |entry| of each row half of each stored tile
  double* rsum;
  double* obs;       // [0..2] S_XX, S_YY, S_XY; [3] observed statistic; [4] R;
                     // [5] power-of-two scale of the fp16 planes
  void* planes;
  uint32_t* Z;
  double* part;
  double* pstat;
  int32_t* flags;    // [0] non-finite input seen, [1] refined pair count, [FLAG_XMAX] max |x|
  // flags[FLAG_COUNT..+1]: exceedance count (low half) and finished workgroups (high half)
  double* perm_out;
  DevResult* result;
  // Asynchronous single-test calls: the caller's result buffer, which the final kernel
  // fills with the result's leading six words (the etest_result fields) beside *result
  // (NULL: none).
  double* out6;
  // Shared block stage: an energy-distance test whose Gram also yields the Gaussian-kernel
  // blocks of an MMD test on the same data (pD != nullptr) writes that test's D, tile sums,
  // tile max and flags too.
  void* pD;
  double* ptsum;
  float* ptmax;
  int32_t* pflags;
  double pgamma;
  // Cross tests (cross-MMD / cross-ED): x and y are cut in halves and staged as the
  // "x side" [x1; y1] (nx = cnx1 + cny1 rows) and the "y side" [x2; y2]; only the
  // rectangle of tiles x side by y side is computed, and each tile keeps its row sums over
  // the x2 columns and over the y2 columns apart.
  int32_t cross, cnx1, cny1, cnx2;
  // Dense pooled matrix (the pre-computation test as the paper prints it): every tile
  // (i, j) of the nt x nt grid, row-major (tile i * nt + j), both orders of every pair.
  int32_t dense;
  // Standard permutation test: staging position t reads pooled item rowmap[t] (x* items in
  // increasing order, then y* items), so one split's X* and Y* are staged without copying
  // the data; NULL reads the items in their own order.
  const int32_t* rowmap;
};

// Input row t of the pooled sample, in staging order: x rows then y rows (through the
// row map when there is one); for a cross test x1, y1, x2, y2.
template <typename T>
__device__ inline const T* pooled_row(const TestDesc& d, int64_t t) {
  const T* X = (const T*)d.X;
  const T* Y = (const T*)d.Y;
  if (!d.cross) {
    if (d.rowmap) t = d.rowmap[t];
    return t < d.nx ? X + t * d.p : Y + (t - d.nx) * d.p;
  }
  if (t < d.cnx1) return X + t * d.p;
  t -= d.cnx1;
  if (t < d.cny1) return Y + t * d.p;
  t -= d.cny1;
  if (t < d.cnx2) return X + (d.cnx1 + t) * d.p;
  return Y + (d.cny1 + t - d.cnx2) * d.p;
}

// Workgroups of a launch are dealt to the 8 XCDs in turn (workgroup b on XCD b % 8), and
// each XCD has its own L2.  xcd_grouped renumbers them so that every XCD works through
// runs of XCD_GROUP consecutive units of the flattened work list (neighbouring units read
// the same operand tiles and then share an L2), while the runs themselves are still dealt
// to the XCDs in turn, which keeps their loads balanced.  A bijection on [0, grid): the
// tail that does not fill a whole round of 8 runs keeps its order.
constexpr int NUM_XCD = 8;
constexpr int XCD_GROUP = 8;
__device__ inline int64_t xcd_grouped(int64_t bid, int64_t grid) {
  const int64_t round = (int64_t)NUM_XCD * XCD_GROUP;
  if (bid >= grid / round * round) return bid;
  const int64_t x = bid % NUM_XCD, k = bid / NUM_XCD;
  return ((k / XCD_GROUP) * NUM_XCD + x) * XCD_GROUP + k % XCD_GROUP;
}

// Staging grids.  Partial column sums: one thread per (row chunk, column); for p < 256 a
// 256-thread workgroup covers 256 / p row chunks of all p columns (otherwise most of its
// threads would idle at small p), for p >= 256 one row chunk of 256 columns.
__host__ __device__ inline int colpart_chunks_per_wg(int64_t p) {
  return p >= 256 ? 1 : (int)(256 / p);
}
__host__ __device__ inline int64_t colpart_wgs(int64_t nrowchunks, int64_t p) {
  const int c = colpart_chunks_per_wg(p);
  return p >= 256 ? nrowchunks * ((p + 255) / 256) : (nrowchunks + c - 1) / c;
}
// Operand staging: the lanes that stage one padded row, the power of two covering p_pad / 4
// (four columns per lane) up to a whole wave, so that a wave stages 64 / that many rows.
__host__ __device__ inline int stage_lanes_per_row(int64_t p_pad) {
  int l = 1;
  while (l < 64 && 4 * l < p_pad) l <<= 1;
  return l;
}
__host__ __device__ inline int64_t stage_wgs(int64_t npad, int64_t p_pad) {
  const int64_t rows = 4 * (64 / stage_lanes_per_row(p_pad));  // per 4-wave workgroup
  return (npad + rows - 1) / rows;
}

// Which test a flattened workgroup index belongs to: offs[t] <= bid < offs[t+1].
__device__ inline int find_test(const int64_t* __restrict__ offs, int ntests, int64_t bid) {
  int lo = 0, hi = ntests - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Stored upper tile index of (i, j), i <= j, in an nt x nt tile grid (formed in 64 bits;
// below 2^31 whenever nt <= MAX_TILE_GRID).
__host__ __device__ inline int64_t tile_index(int i, int j, int nt) {
  const int64_t a = i;
  return a * nt - (a * (a - 1)) / 2 + (j - i);
}

// Inverse of tile_index.
__device__ inline void tile_coords(int t, int nt, int* pi, int* pj) {
  int i = 0;
  int start = 0;
  while (true) {
    int len = nt - i;
    if (t < start + len) break;
    start += len;
    ++i;
  }
  *pi = i;
  *pj = i + (t - start);
}

// Real rows in pooled tile i (rest is padding).
__device__ inline int tile_rows(const TestDesc& d, int i) {
  if (i < d.tx) {
    int r = d.nx - i * TILE;
    return r < TILE ? r : TILE;
  }
  int r = d.ny - (i - d.tx) * TILE;
  return r < TILE ? r : TILE;
}

// Row unit u of a test -> (row tile i, column tiles [j0, j1)).  Row i holds the stored
// tiles j = i .. nt-1 cut into ceil((nt - i) / kc) units of kc tiles (the last one shorter);
// units are numbered row by row.  The walk over rows uses no division inside the loop: with
// q = nt - i, the unit count ceil(q / kc) drops by one exactly when (q - 1) % kc was 0.
__host__ __device__ inline void rowk_coords(const TestDesc& d, int u, int* pi, int* pj0,
                                            int* pj1) {
  const int kc = d.kc;
  int i = 0, start = 0;
  int len = (d.nt + kc - 1) / kc, r = (d.nt - 1) % kc;
  while (u >= start + len) {
    start += len;
    ++i;
    if (r == 0) {
      --len;
      r = kc - 1;
    } else {
      --r;
    }
  }
  *pi = i;
  *pj0 = i + (u - start) * kc;
  const int e = *pj0 + kc;
  *pj1 = e < d.nt ? e : d.nt;
}

// FP32 -> fp8 E4M3 in the OCP layout the gfx950 fp8 MFMA reads (bias 7, no infinities,
// 0x7F / 0xFF are NaN, largest finite 448): round to nearest even, saturating at +-448;
// subnormals (multiples of 2^-9) kept.  Finite inputs only; zero of either sign -> 0.
__host__ __device__ inline uint32_t f32_to_e4m3(float x) {
  const uint32_t sign = (__builtin_bit_cast(uint32_t, x) >> 24) & 0x80u;
  const float a = __builtin_fabsf(x);
  uint32_t code;
  if (a < 0.015625f) {
    // below 2^-6: multiples of 2^-9; code 8 (2^-6, the smallest normal) follows on
    code = (uint32_t)__builtin_rintf(a * 512.0f);
  } else {
    uint32_t ua = __builtin_bit_cast(uint32_t, a);
    ua += 0x7FFFFu + ((ua >> 20) & 1u);  // 23-bit mantissa -> 3 bits, nearest even
    const uint32_t e = (ua >> 23) - 120u;  // exponent rebiased from 127 to 7
    code = e > 15u ? 0x7Eu : ((e << 3) | ((ua >> 20) & 7u));
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return code ? (sign | code) : 0u;
}

// FP32 form: the centred operand w is staged as two fp16 values per entry, hi = fp16(w 2^e)
// and lo = fp16(w 2^e - hi) (together 22 significant bits; every product of two of them is
// exact in FP32).  max |x| over the input bounds every centred value by 2 max|x| < 2^(ex+1)
// (max|x| = m 2^ex, 0.5 <= m < 1), so e = 13 - ex keeps |w 2^e| below 2^14, inside fp16's
// range.  Returns e (0 without a finite positive maximum).
__device__ inline int f16_split_exponent(const TestDesc& d) {
  const float m = __uint_as_float((uint32_t)d.flags[FLAG_XMAX]);
  if (!(m > 0.0f) || !isfinite(m)) return 0;
  int ex;
  (void)frexpf(m, &ex);
  const int e = 13 - ex;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4 x 32 S-box with
// the published multipliers and Weyl key increments.  Counter c, key (k0, k1).
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__device__ inline uint16_t f32_to_bf16_rn(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)((u + r) >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

}  // namespace et
