/*
 * FP64 CPU oracle for the Hines solve.  TEST INFRASTRUCTURE ONLY: tests, the
 * smoke check and the bench's CPU-baseline leg use it; the library never does.
 * It shares no code, header or table with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * IEEE division), so each operation below is one rounded FP64 operation.
 *
 * Conventions (paper §1, the discrete implicit-Euler system; §2, the arrays
 * d, u, b, p of the Hines algorithm), user numbering:
 *   cell c owns compartments [cell_off[c], cell_off[c+1]); its first
 *   compartment is the root (parent -1); every other i has
 *   cell_off[c] <= p[i] < i.
 *   d[i] = A[i][i];  u[i] = A[i][p[i]] = A[p[i]][i] (signed entry; symmetric A).
 * Reading of the paper's listings: the coupling of compartment i to its parent
 * is u[i] in BOTH sweeps (§2 says u stores "the coupling entries to the parent
 * of a compartment"); the printed backward loop indexes it by the parent,
 * which does not solve the system.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* One cell of the Hines algorithm (paper §2, Listing 2 with the index reading
 * above): backward elimination from the last compartment to the root through
 * p[], root solve, forward substitution from the root.  d is overwritten by the
 * eliminated diagonal, b by the solution.  Returns the number of pivots that
 * were not strictly positive (0 for a strictly diagonally dominant matrix with
 * positive diagonal, paper §1). */
static int64_t hines_cell_f64(int64_t lo, int64_t hi, const int32_t *p, double *d,
                              const double *u, double *b) {
  int64_t bad = 0;
  for (int64_t i = hi - 1; i > lo; --i) {
    if (!(d[i] > 0.0)) ++bad;
    double f = u[i] / d[i];
    d[p[i]] = d[p[i]] - f * u[i];
    b[p[i]] = b[p[i]] - f * b[i];
  }
  if (!(d[lo] > 0.0)) ++bad;
  b[lo] = b[lo] / d[lo];
  for (int64_t i = lo + 1; i < hi; ++i) b[i] = (b[i] - u[i] * b[p[i]]) / d[i];
  return bad;
}

/* The same algorithm carried out in FP32 (used by the refinement oracle). */
static int64_t hines_cell_f32(int64_t lo, int64_t hi, const int32_t *p, float *d,
                              const float *u, float *b) {
  int64_t bad = 0;
  for (int64_t i = hi - 1; i > lo; --i) {
    if (!(d[i] > 0.0f)) ++bad;
    float f = u[i] / d[i];
    d[p[i]] = d[p[i]] - f * u[i];
    b[p[i]] = b[p[i]] - f * b[i];
  }
  if (!(d[lo] > 0.0f)) ++bad;
  b[lo] = b[lo] / d[lo];
  for (int64_t i = lo + 1; i < hi; ++i) b[i] = (b[i] - u[i] * b[p[i]]) / d[i];
  return bad;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* Solve A x = b for every cell (cells are independent, paper §3).
 * d and b are overwritten (d: eliminated diagonal, b: x).  Returns the total
 * count of non-positive pivots. */
int64_t oracle_solve_f64(int64_t ncells, const int64_t *cell_off, const int32_t *p, double *d,
                         const double *u, double *b, int nthreads) {
  int64_t bad = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t c = 0; c < ncells; ++c) bad += hines_cell_f64(cell_off[c], cell_off[c + 1], p, d, u, b);
  return bad;
}

int64_t oracle_solve_f32(int64_t ncells, const int64_t *cell_off, const int32_t *p, float *d,
                         const float *u, float *b, int nthreads) {
  int64_t bad = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t c = 0; c < ncells; ++c) bad += hines_cell_f32(cell_off[c], cell_off[c + 1], p, d, u, b);
  return bad;
}

/* y = A x for the tree matrix defined by (d, u, p): row i holds d[i] on the
 * diagonal, u[i] at column p[i], and u[k] at column k for every child k of i
 * (symmetry, paper §1).  Per cell, sequential, fixed order. */
void oracle_spmv_f64(int64_t ncells, const int64_t *cell_off, const int32_t *p, const double *d,
                     const double *u, const double *x, double *y, int nthreads) {
  set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < ncells; ++c) {
    int64_t lo = cell_off[c], hi = cell_off[c + 1];
    for (int64_t i = lo; i < hi; ++i) y[i] = d[i] * x[i];
    for (int64_t i = lo + 1; i < hi; ++i) {
      y[i] = y[i] + u[i] * x[p[i]];
      y[p[i]] = y[p[i]] + u[i] * x[i];
    }
  }
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of the two 32x32->64 multiplications
 * with the published multipliers and Weyl key increments. */
static void philox4x32_10(uint32_t ctr[4], const uint32_t key_in[2]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * ctr[0];
    uint64_t p1 = (uint64_t)M1 * ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ k0;
    uint32_t n2 = hi0 ^ ctr[3] ^ k1;
    ctr[0] = n0; ctr[1] = lo1; ctr[2] = n2; ctr[3] = lo0;
  }
}

void oracle_philox(const uint32_t *ctr_in, const uint32_t *key, uint32_t *out) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  philox4x32_10(c, key);
  memcpy(out, c, sizeof c);
}

/* Injected-current draws of the time loop: out[j] = scale * Z with Z standard
 * normal from Box-Muller on two 52-bit uniforms of one Philox block keyed by
 * (seed, 0) with counter (idx lo, idx hi, step, 0).  idx is the user index, so
 * a draw does not depend on any solver layout. */
void oracle_noise(uint32_t seed, uint32_t step, int64_t count, const int64_t *idx, double scale,
                  double *out) {
  const double two_pi = 6.283185307179586476925286766559;
  const double ulp52 = 1.0 / 4503599627370496.0; /* 2^-52 */
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < count; ++j) {
    uint64_t i = (uint64_t)idx[j];
    uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), step, 0u};
    uint32_t k[2] = {seed, 0u};
    philox4x32_10(c, k);
    uint64_t m1 = (((uint64_t)c[0] << 32) | c[1]) >> 12;
    uint64_t m2 = (((uint64_t)c[2] << 32) | c[3]) >> 12;
    double u1 = ((double)m1 + 0.5) * ulp52;
    double u2 = ((double)m2 + 0.5) * ulp52;
    out[j] = scale * (sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
  }
}
