/*
 * FP64 CPU oracle for the efficient permutation two-sample test
 * (Chaibub Neto, arXiv 2406.06488).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do. It shares no code, header, table or constant with the
 * HIP path.
 *
 * Everything here is plain and slow on purpose:
 *   - distance / kernel blocks by direct differences (Alg. 3 and the
 *     Gaussian-kernel remark that follows it, Appendix A.1);
 *   - observed statistic by eq. (1) (energy distance) or eq. (2) (biased
 *     MMD^2) over the full blocks;
 *   - each resampled statistic by filling the three permuted blocks from the
 *     four sub-blocks of D_XX, D_XY, D_YX = D_XY^T and D_YY named by the index
 *     vectors i1, i2, j1, j2 of Alg. 2 (Alg. 1 "for" loop, with the
 *     memory-saving transposed read described after Alg. 1), then averaging
 *     them as eq. (1) / eq. (2) prescribe;
 *   - p-value (1 + #{stat* >= stat_o}) / (1 + b)  (Section 3.1, Phipson-Smyth).
 *
 * Readings where the paper leaves a choice:
 *   - every block sum is exactly rounded (Shewchuk expansion plus a final
 *     correctly rounded collapse), so a statistic is a function of the split
 *     as a set, independent of summation order;
 *   - the counting threshold is the identity split evaluated by the same code
 *     that evaluates each resampled split (it equals eq. (1)/(2) exactly,
 *     because the sums are exact);
 *   - the paper draws splits with R's sample(); here split b is drawn by
 *     selection sampling (Knuth, TAOCP vol. 2, 3.4.2, Algorithm S) driven by
 *     Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key = seed and
 *     counter = (t/2, b_lo, b_hi, 0): any exactly uniform subset sampler
 *     gives a valid permutation test, and the statistic depends only on the
 *     chosen subset (Appendix A.4, last paragraph);
 *   - Gaussian kernel k(x, y) = exp(-gamma * ||x - y||^2) with gamma = 1/sigma^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ED 0
#define ORC_MMD 1

/* ------------------------------------------------------------------------- */
/* Exactly rounded summation.                                                 */
/* Partials form a non-overlapping expansion (Shewchuk 1997, Grow-Expansion   */
/* with zero elimination); the collapse rounds the exact value once, with the */
/* round-half-even fix-up when the discarded tail sits exactly at a half ulp. */
/* ------------------------------------------------------------------------- */
typedef struct {
  double p[80];
  int n;
} xacc;

static void xacc_init(xacc* a) { a->n = 0; }

static void xacc_add(xacc* a, double x) {
  int keep = 0;
  for (int j = 0; j < a->n; j++) {
    double y = a->p[j];
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;          /* TwoSum with |x| >= |y|: exact split */
    double lo = y - (hi - x);
    if (lo != 0.0) a->p[keep++] = lo;
    x = hi;
  }
  if (keep >= 80) abort(); /* cannot happen for finite doubles */
  a->p[keep++] = x;
  a->n = keep;
}

static double xacc_value(const xacc* a) {
  int n = a->n;
  if (n == 0) return 0.0;
  double hi = a->p[--n];
  double lo = 0.0;
  while (n > 0) {
    double x = hi;
    double y = a->p[--n];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  /* The tail below 'lo' decides a tie: if lo is exactly half an ulp of hi and
     the remaining partials push further in the same direction, round away. */
  if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

double orc_xsum(const double* v, int64_t n) {
  xacc a;
  xacc_init(&a);
  for (int64_t i = 0; i < n; i++) xacc_add(&a, v[i]);
  return xacc_value(&a);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 S-box with the */
/* published multipliers and Weyl key increments.                             */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64-bit uniform draw for pooled item t of split b. */
static uint64_t draw_u64(uint64_t seed, uint64_t b, uint64_t t) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(t >> 1), (uint32_t)b, (uint32_t)(b >> 32), 0u};
  uint32_t r[4];
  orc_philox4x32_10(ctr, key, r);
  if (t & 1u) return ((uint64_t)r[3] << 32) | r[2];
  return ((uint64_t)r[1] << 32) | r[0];
}

/* Split b: z[t] = 1 when pooled item t (X rows 0..nx-1, then Y rows) goes to
   x*.  Selection sampling keeps item t with probability need / (n - t),
   decided in integers as floor(u * (n - t) / 2^64) < need. */
int orc_membership(int64_t nx, int64_t ny, uint64_t seed, int64_t b, uint8_t* z) {
  if (nx < 1 || ny < 1 || b < 0 || !z) return 1;
  int64_t n = nx + ny, need = nx;
  for (int64_t t = 0; t < n; t++) {
    uint64_t m = (uint64_t)(n - t);
    uint64_t u = draw_u64(seed, (uint64_t)b, (uint64_t)t);
    uint64_t v = (uint64_t)(((unsigned __int128)u * m) >> 64);
    uint8_t take = v < (uint64_t)need ? 1 : 0;
    z[t] = take;
    need -= take;
  }
  return 0;
}

/* Alg. 2, from a membership vector: i1 = X rows in x*, i2 = Y rows in x*,
   j1 = X rows in y*, j2 = Y rows in y* (0-based, ascending). */
int orc_split_indices(int64_t nx, int64_t ny, const uint8_t* z, int64_t* i1, int64_t* i2,
                      int64_t* j1, int64_t* j2, int64_t counts[4]) {
  int64_t a = 0, b = 0, c = 0, d = 0;
  for (int64_t t = 0; t < nx; t++) {
    if (z[t]) i1[a++] = t;
    else j1[c++] = t;
  }
  for (int64_t t = 0; t < ny; t++) {
    if (z[nx + t]) i2[b++] = t;
    else j2[d++] = t;
  }
  counts[0] = a; counts[1] = b; counts[2] = c; counts[3] = d;
  return 0;
}

/* Alg. 3: D[i][j] = (sum_k (a_ik - b_jk)^2)^(1/2); for the Gaussian kernel
   K[i][j] = exp(-gamma * sum_k (a_ik - b_jk)^2). */
int orc_block(const double* A, int64_t na, const double* Bm, int64_t nb, int64_t p, int kind,
              double gamma, double* out, int nthreads) {
  if (na < 1 || nb < 1 || p < 1) return 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < na; i++) {
    for (int64_t j = 0; j < nb; j++) {
      double s = 0.0;
      for (int64_t k = 0; k < p; k++) {
        double d = A[i * p + k] - Bm[j * p + k];
        s += d * d;
      }
      out[i * nb + j] = (kind == ORC_ED) ? sqrt(s) : exp(-gamma * s);
    }
  }
  return 0;
}

/* Combine the three block averages.  ED  (eq. 1) = 2/(nx ny) S_xy - S_xx/nx^2 - S_yy/ny^2;
   MMD (eq. 2) = S_xx/nx^2 + S_yy/ny^2 - 2/(nx ny) S_xy.  The three terms are
   added exactly and rounded once, so the result does not depend on which
   group is called x. */
static double combine(int kind, double sxx, double syy, double sxy, int64_t nx, int64_t ny) {
  double txy = (2.0 * sxy) / ((double)nx * (double)ny);
  double txx = sxx / ((double)nx * (double)nx);
  double tyy = syy / ((double)ny * (double)ny);
  xacc a;
  xacc_init(&a);
  if (kind == ORC_ED) {
    xacc_add(&a, txy);
    xacc_add(&a, -txx);
    xacc_add(&a, -tyy);
  } else {
    xacc_add(&a, txx);
    xacc_add(&a, tyy);
    xacc_add(&a, -txy);
  }
  return xacc_value(&a);
}

/* Observed statistic from the blocks (Alg. 1 line computing ED_o). */
int orc_observed(int kind, const double* XX, const double* YY, const double* XY, int64_t nx,
                 int64_t ny, double* stat, double sums[3]) {
  double sxx = orc_xsum(XX, nx * nx);
  double syy = orc_xsum(YY, ny * ny);
  double sxy = orc_xsum(XY, nx * ny);
  if (sums) {
    sums[0] = sxx; sums[1] = syy; sums[2] = sxy;
  }
  *stat = combine(kind, sxx, syy, sxy, nx, ny);
  return 0;
}

/* One resampled statistic (Alg. 1 loop body): the permuted blocks are filled
   from the original ones,
     D_{X*X*} = [ D_XX[i1,i1]  D_XY[i1,i2] ; D_YX[i2,i1]  D_YY[i2,i2] ]
     D_{Y*Y*} = [ D_XX[j1,j1]  D_XY[j1,j2] ; D_YX[j2,j1]  D_YY[j2,j2] ]
     D_{X*Y*} = [ D_XX[i1,j1]  D_XY[i1,j2] ; D_YX[i2,j1]  D_YY[i2,j2] ]
   with D_YX[r,c] read as D_XY[c,r], and only their element sums are kept. */
static void perm_sums_idx(const double* XX, const double* YY, const double* XY, int64_t nx,
                          int64_t ny, const int64_t* i1, int64_t n1, const int64_t* i2,
                          int64_t n2, const int64_t* j1, int64_t m1, const int64_t* j2,
                          int64_t m2, double out[3]) {
  xacc sxx, syy, sxy;
  xacc_init(&sxx);
  xacc_init(&syy);
  xacc_init(&sxy);
  /* D_{X*X*} */
  for (int64_t r = 0; r < n1; r++)
    for (int64_t c = 0; c < n1; c++) xacc_add(&sxx, XX[i1[r] * nx + i1[c]]);
  for (int64_t r = 0; r < n1; r++)
    for (int64_t c = 0; c < n2; c++) xacc_add(&sxx, XY[i1[r] * ny + i2[c]]);
  for (int64_t r = 0; r < n2; r++)
    for (int64_t c = 0; c < n1; c++) xacc_add(&sxx, XY[i1[c] * ny + i2[r]]);
  for (int64_t r = 0; r < n2; r++)
    for (int64_t c = 0; c < n2; c++) xacc_add(&sxx, YY[i2[r] * ny + i2[c]]);
  /* D_{Y*Y*} */
  for (int64_t r = 0; r < m1; r++)
    for (int64_t c = 0; c < m1; c++) xacc_add(&syy, XX[j1[r] * nx + j1[c]]);
  for (int64_t r = 0; r < m1; r++)
    for (int64_t c = 0; c < m2; c++) xacc_add(&syy, XY[j1[r] * ny + j2[c]]);
  for (int64_t r = 0; r < m2; r++)
    for (int64_t c = 0; c < m1; c++) xacc_add(&syy, XY[j1[c] * ny + j2[r]]);
  for (int64_t r = 0; r < m2; r++)
    for (int64_t c = 0; c < m2; c++) xacc_add(&syy, YY[j2[r] * ny + j2[c]]);
  /* D_{X*Y*} */
  for (int64_t r = 0; r < n1; r++)
    for (int64_t c = 0; c < m1; c++) xacc_add(&sxy, XX[i1[r] * nx + j1[c]]);
  for (int64_t r = 0; r < n1; r++)
    for (int64_t c = 0; c < m2; c++) xacc_add(&sxy, XY[i1[r] * ny + j2[c]]);
  for (int64_t r = 0; r < n2; r++)
    for (int64_t c = 0; c < m1; c++) xacc_add(&sxy, XY[j1[c] * ny + i2[r]]);
  for (int64_t r = 0; r < n2; r++)
    for (int64_t c = 0; c < m2; c++) xacc_add(&sxy, YY[i2[r] * ny + j2[c]]);
  out[0] = xacc_value(&sxx);
  out[1] = xacc_value(&syy);
  out[2] = xacc_value(&sxy);
}

/* Element sums of the permuted blocks D_{X*X*}, D_{Y*Y*}, D_{X*Y*} for split z. */
int orc_perm_sums(const double* XX, const double* YY, const double* XY, int64_t nx, int64_t ny,
                  const uint8_t* z, double sums[3]) {
  int64_t n = nx + ny, cnt = 0;
  for (int64_t t = 0; t < n; t++) cnt += z[t] ? 1 : 0;
  if (cnt != nx) return 1;
  /* i1 (<= nx), i2 (<= ny), j1 (<= nx), j2 (<= ny): separate ranges. */
  int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * n));
  if (!buf) return 3;
  int64_t *i1 = buf, *i2 = buf + nx, *j1 = buf + n, *j2 = buf + n + nx;
  int64_t counts[4];
  orc_split_indices(nx, ny, z, i1, i2, j1, j2, counts);
  perm_sums_idx(XX, YY, XY, nx, ny, i1, counts[0], i2, counts[1], j1, counts[2], j2, counts[3],
                sums);
  free(buf);
  return 0;
}

int orc_perm_stat(int kind, const double* XX, const double* YY, const double* XY, int64_t nx,
                  int64_t ny, const uint8_t* z, double* stat) {
  double sums[3];
  int r = orc_perm_sums(XX, YY, XY, nx, ny, z, sums);
  if (r) return r;
  *stat = combine(kind, sums[0], sums[1], sums[2], nx, ny);
  return 0;
}

/* Resampled statistics for the listed splits b (membership drawn from
   (seed, b)), computed one by one from the given blocks. */
int orc_perm_stats_listed(int kind, const double* XX, const double* YY, const double* XY,
                          int64_t nx, int64_t ny, uint64_t seed, const int64_t* b_list,
                          int64_t n_list, double* out, int nthreads) {
  int64_t n = nx + ny;
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    uint8_t* z = (uint8_t*)malloc((size_t)n);
    if (!z) {
#pragma omp atomic write
      err = 3;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < n_list; i++) {
        orc_membership(nx, ny, seed, b_list[i], z);
        if (orc_perm_stat(kind, XX, YY, XY, nx, ny, z, &out[i]) != 0) {
#pragma omp atomic write
          err = 3;
        }
      }
      free(z);
    }
  }
  return err;
}

/* Identity split: x* = x, y* = y. */
int orc_threshold(int kind, const double* XX, const double* YY, const double* XY, int64_t nx,
                  int64_t ny, double* thr) {
  int64_t n = nx + ny;
  uint8_t* z = (uint8_t*)malloc((size_t)n);
  if (!z) return 3;
  for (int64_t t = 0; t < n; t++) z[t] = t < nx ? 1 : 0;
  int r = orc_perm_stat(kind, XX, YY, XY, nx, ny, z, thr);
  free(z);
  return r;
}

/* Full test (Alg. 1): blocks once, observed statistic, B resampled
   statistics, threshold, exceedance count and p-value.  The caller may
   provide the three blocks (computed with orc_block) to avoid recomputing. */
int orc_test(int kind, const double* X, int64_t nx, const double* Y, int64_t ny, int64_t p,
             double gamma, int64_t B, uint64_t seed, double* perm_stats, double* stat_obs,
             double* threshold, int64_t* count_ge, double* p_value, int nthreads) {
  if (nx < 1 || ny < 1 || p < 1 || B < 0) return 1;
  if (kind == ORC_MMD && !(gamma > 0.0)) return 1;
  double* XX = (double*)malloc(sizeof(double) * (size_t)(nx * nx));
  double* YY = (double*)malloc(sizeof(double) * (size_t)(ny * ny));
  double* XY = (double*)malloc(sizeof(double) * (size_t)(nx * ny));
  int64_t* bl = (int64_t*)malloc(sizeof(int64_t) * (size_t)(B > 0 ? B : 1));
  double* ps = perm_stats ? perm_stats : (double*)malloc(sizeof(double) * (size_t)(B > 0 ? B : 1));
  int r = 0;
  if (!XX || !YY || !XY || !bl || !ps) {
    r = 3;
    goto done;
  }
  orc_block(X, nx, X, nx, p, kind, gamma, XX, nthreads);
  orc_block(Y, ny, Y, ny, p, kind, gamma, YY, nthreads);
  orc_block(X, nx, Y, ny, p, kind, gamma, XY, nthreads);
  orc_observed(kind, XX, YY, XY, nx, ny, stat_obs, NULL);
  r = orc_threshold(kind, XX, YY, XY, nx, ny, threshold);
  if (r) goto done;
  for (int64_t b = 0; b < B; b++) bl[b] = b;
  r = orc_perm_stats_listed(kind, XX, YY, XY, nx, ny, seed, bl, B, ps, nthreads);
  if (r) goto done;
  {
    int64_t c = 0;
    for (int64_t b = 0; b < B; b++) c += (ps[b] >= *threshold) ? 1 : 0;
    *count_ge = c;
    *p_value = (1.0 + (double)c) / (1.0 + (double)B);
  }
done:
  free(XX);
  free(YY);
  free(XY);
  free(bl);
  if (ps != perm_stats) free(ps);
  return r;
}

/* ------------------------------------------------------------------------- */
/* Cross-MMD test (Alg. 6) and cross-ED test (Alg. 7), appendix "The cross-ED  */
/* test".  x is cut into x1 (its first floor(nx/2) rows) and x2 (the rest), y  */
/* likewise; the four cross blocks come from orc_block (direct differences).   */
/*   MMD: U_x = mean K(x1,x2) - mean K(x1,y2),  U_y = mean K(y1,x2) - mean K(y1,y2) */
/*   ED:  U_x = mean D(x1,y2) - mean D(x1,x2),  U_y = mean D(y1,y2) - mean D(y1,x2) */
/*   U = U_x - U_y;  s_x = mean over x1 rows of (row mean difference - U_x)^2,     */
/*   s_y likewise over y1 rows;  sigma = sqrt(s_x / nx1 + s_y / ny1);              */
/*   p = 1 - Phi(U / sigma), written as erfc(z / sqrt 2) / 2 so that the upper     */
/*   tail keeps its digits.  Every mean is an exactly rounded sum (orc_xsum)        */
/*   divided by its count.                                                          */
/* Reading: sigma = 0 gives z = +inf, -inf or 0 by the sign of U (p = 0, 1, 1/2).   */
/* out[0] = U, out[1] = sigma, out[2] = z, out[3] = p.                               */
/* ------------------------------------------------------------------------- */
static double mean_of(const double* v, int64_t n) { return orc_xsum(v, n) / (double)n; }

/* mean over the rows of (row mean of A - row mean of B - u)^2; A is rows x na, B rows x nb */
static double row_spread(const double* A, int64_t na, const double* Bm, int64_t nb, int64_t rows,
                         double u) {
  double* d2 = (double*)malloc(sizeof(double) * (size_t)rows);
  if (!d2) return NAN;
  for (int64_t i = 0; i < rows; i++) {
    double f = mean_of(A + i * na, na) - mean_of(Bm + i * nb, nb) - u;
    d2[i] = f * f;
  }
  double s = mean_of(d2, rows);
  free(d2);
  return s;
}

int orc_cross(int kind, const double* X, int64_t nx, const double* Y, int64_t ny, int64_t p,
              double gamma, double out[4], int nthreads) {
  if (nx < 2 || ny < 2 || p < 1) return 1;
  if (kind == ORC_MMD && !(gamma > 0.0)) return 1;
  const int64_t nx1 = nx / 2, nx2 = nx - nx1, ny1 = ny / 2, ny2 = ny - ny1;
  const double* x1 = X;
  const double* x2 = X + nx1 * p;
  const double* y1 = Y;
  const double* y2 = Y + ny1 * p;
  double* KX1X2 = (double*)malloc(sizeof(double) * (size_t)(nx1 * nx2));
  double* KY1Y2 = (double*)malloc(sizeof(double) * (size_t)(ny1 * ny2));
  double* KX1Y2 = (double*)malloc(sizeof(double) * (size_t)(nx1 * ny2));
  double* KY1X2 = (double*)malloc(sizeof(double) * (size_t)(ny1 * nx2));
  int r = 0;
  if (!KX1X2 || !KY1Y2 || !KX1Y2 || !KY1X2) {
    r = 3;
    goto done;
  }
  orc_block(x1, nx1, x2, nx2, p, kind, gamma, KX1X2, nthreads);
  orc_block(y1, ny1, y2, ny2, p, kind, gamma, KY1Y2, nthreads);
  orc_block(x1, nx1, y2, ny2, p, kind, gamma, KX1Y2, nthreads);
  orc_block(y1, ny1, x2, nx2, p, kind, gamma, KY1X2, nthreads);
  {
    /* the block whose mean enters with + and the one with -, for x1 rows and y1 rows */
    const int ed = kind == ORC_ED;
    const double* xa = ed ? KX1Y2 : KX1X2;
    const double* xb = ed ? KX1X2 : KX1Y2;
    const int64_t na = ed ? ny2 : nx2, nb = ed ? nx2 : ny2;
    const double* ya = ed ? KY1Y2 : KY1X2;
    const double* yb = ed ? KY1X2 : KY1Y2;
    const int64_t ma = ed ? ny2 : nx2, mb = ed ? nx2 : ny2;
    const double ux = mean_of(xa, nx1 * na) - mean_of(xb, nx1 * nb);
    const double uy = mean_of(ya, ny1 * ma) - mean_of(yb, ny1 * mb);
    const double u = ux - uy;
    const double sx = row_spread(xa, na, xb, nb, nx1, ux);
    const double sy = row_spread(ya, ma, yb, mb, ny1, uy);
    const double sigma = sqrt(sx / (double)nx1 + sy / (double)ny1);
    double z;
    if (sigma > 0.0) z = u / sigma;
    else z = u > 0.0 ? INFINITY : (u < 0.0 ? -INFINITY : 0.0);
    out[0] = u;
    out[1] = sigma;
    out[2] = z;
    out[3] = 0.5 * erfc(z / sqrt(2.0));
  }
done:
  free(KX1X2);
  free(KY1Y2);
  free(KX1Y2);
  free(KY1X2);
  return r;
}

/* ------------------------------------------------------------------------- */
/* HSIC independence permutation test: the extension the paper's discussion   */
/* proposes (Gretton et al. 2007), with the unbiased HSIC estimator of Song   */
/* et al. (2012) that the discussion writes out. x_i and y_i are paired; the  */
/* permutations reorder the y sample.                                         */
/* Readings:                                                                  */
/*   - the estimator carries the factor 2 on its third term and the scale     */
/*     1/(n (n-3)) of Song et al.'s unbiased form (the printed formula shows  */
/*     1/(n-3) and no 2; the scale cannot move a permutation p-value, the 2   */
/*     is what makes the estimator unbiased);                                 */
/*   - Gaussian kernels exp(-gamma ||a - b||^2) on x and on y, each with its  */
/*     own gamma;                                                             */
/*   - permutation b orders the items 0..n-1 by a 64-bit Philox4x32-10 key    */
/*     (key = seed, counter = (t/2, b_lo, b_hi, 1); even t takes words 0,1,   */
/*     odd t words 2,3, low word first), ties by index: a uniformly random    */
/*     permutation;                                                           */
/*   - the threshold is the identity permutation through the same code, and  */
/*     p = (1 + #{b : HSIC_b >= threshold}) / (1 + B), as for the two-sample  */
/*     test.                                                                  */
/* ------------------------------------------------------------------------- */
static uint64_t perm_key(uint64_t seed, uint64_t b, uint64_t t) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(t >> 1), (uint32_t)b, (uint32_t)(b >> 32), 1u};
  uint32_t r[4];
  orc_philox4x32_10(ctr, key, r);
  if (t & 1u) return ((uint64_t)r[3] << 32) | r[2];
  return ((uint64_t)r[1] << 32) | r[0];
}

typedef struct {
  uint64_t key;
  int64_t idx;
} keyed_item;

static int cmp_keyed(const void* a, const void* b) {
  const keyed_item* x = (const keyed_item*)a;
  const keyed_item* y = (const keyed_item*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

/* Permutation b: perm[i] = the item placed at position i. */
int orc_permutation(int64_t n, uint64_t seed, int64_t b, int64_t* perm) {
  if (n < 1 || b < 0 || !perm) return 1;
  keyed_item* it = (keyed_item*)malloc(sizeof(keyed_item) * (size_t)n);
  if (!it) return 2;
  for (int64_t t = 0; t < n; t++) {
    it[t].key = perm_key(seed, (uint64_t)b, (uint64_t)t);
    it[t].idx = t;
  }
  qsort(it, (size_t)n, sizeof(keyed_item), cmp_keyed);
  for (int64_t t = 0; t < n; t++) perm[t] = it[t].idx;
  free(it);
  return 0;
}

/* Unbiased HSIC of kernel matrices K (n x n, of x) and L (of y), L read through
   the permutation pi (L_pi[i][j] = L[pi_i][pi_j]; pi = NULL for the identity).
   With Kt = K - diag(K) and Lt = L - diag(L):
     T1 = tr(Kt Lt_pi) = sum_{i != j} K[i][j] L[pi_i][pi_j]
     T2 = (1^T Kt 1)(1^T Lt 1)
     T3 = 1^T Kt Lt_pi 1 = sum_i (Kt 1)_i (Lt 1)_{pi_i}
     HSIC = [T1 + T2 / ((n-1)(n-2)) - 2 T3 / (n-2)] / (n (n-3)).
   Every sum is exactly rounded. */
static double hsic_value(const double* K, const double* L, int64_t n, const int64_t* pi) {
  xacc t1, sk, sl, t3;
  xacc_init(&t1);
  xacc_init(&sk);
  xacc_init(&sl);
  xacc_init(&t3);
  double* rk = (double*)malloc(sizeof(double) * (size_t)n);
  double* rl = (double*)malloc(sizeof(double) * (size_t)n);
  if (!rk || !rl) {
    free(rk);
    free(rl);
    return NAN;
  }
  for (int64_t i = 0; i < n; i++) {
    xacc a, c;
    xacc_init(&a);
    xacc_init(&c);
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      xacc_add(&a, K[i * n + j]);
      xacc_add(&c, L[i * n + j]);
    }
    rk[i] = xacc_value(&a);
    rl[i] = xacc_value(&c);
  }
  for (int64_t i = 0; i < n; i++) {
    const int64_t pii = pi ? pi[i] : i;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      const int64_t pj = pi ? pi[j] : j;
      xacc_add(&t1, K[i * n + j] * L[pii * n + pj]);
      xacc_add(&sk, K[i * n + j]);
      xacc_add(&sl, L[i * n + j]);
    }
    xacc_add(&t3, rk[i] * rl[pii]);
  }
  const double dn = (double)n;
  const double T1 = xacc_value(&t1), T2 = xacc_value(&sk) * xacc_value(&sl), T3 = xacc_value(&t3);
  free(rk);
  free(rl);
  return (T1 + T2 / ((dn - 1.0) * (dn - 2.0)) - 2.0 * T3 / (dn - 2.0)) / (dn * (dn - 3.0));
}

/* HSIC of given kernel matrices (pi may be NULL). */
int orc_hsic(const double* K, const double* L, int64_t n, const int64_t* pi, double* out) {
  if (n < 4 || !K || !L || !out) return 1;
  *out = hsic_value(K, L, n, pi);
  return isnan(*out) ? 2 : 0;
}

/* The whole test on data: x (n x p), y (n x q), B permutations of y.
   stats[0..B-1]: HSIC of each permutation; out = {statistic, threshold, p_value};
   *count = #{b : stats[b] >= threshold}. */
int orc_hsic_test(const double* X, const double* Y, int64_t n, int64_t p, int64_t q,
                  double gx, double gy, int64_t B, uint64_t seed, double* stats, double* out,
                  int64_t* count, int nthreads) {
  if (n < 4 || p < 1 || q < 1 || B < 0 || !(gx > 0.0) || !(gy > 0.0) || !out || !count)
    return 1;
  double* K = (double*)malloc(sizeof(double) * (size_t)(n * n));
  double* L = (double*)malloc(sizeof(double) * (size_t)(n * n));
  if (!K || !L) {
    free(K);
    free(L);
    return 2;
  }
  orc_block(X, n, X, n, p, ORC_MMD, gx, K, nthreads);
  orc_block(Y, n, Y, n, q, ORC_MMD, gy, L, nthreads);
  const double thr = hsic_value(K, L, n, NULL);
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int64_t b = 0; b < B; b++) {
    int64_t* pi = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!pi || orc_permutation(n, seed, b, pi)) {
      bad |= 1;
    } else {
      stats[b] = hsic_value(K, L, n, pi);
    }
    free(pi);
  }
  free(K);
  free(L);
  if (bad) return 2;
  int64_t c = 0;
  for (int64_t b = 0; b < B; b++) c += stats[b] >= thr ? 1 : 0;
  out[0] = thr;
  out[1] = thr;
  out[2] = (1.0 + (double)c) / (1.0 + (double)B);
  *count = c;
  return 0;
}
