/*
 * CPU FP64 oracle for the stencil sweep -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never does, and
 * the two share no code: no headers, no helpers, no tables.
 *
 * What it computes (plain definition, no blocking, no reordering):
 *
 *   One Jacobi step (Section 2.2, "Stencil Computation"): the output array B
 *   at time t+1 is computed from the input array A at time t, and the two
 *   arrays swap roles for the next step.
 *
 *   Gather form (Section 3.2, Eq. (1) generalised to order r, with the
 *   (2r+1)^d coefficient tensor C^g of Eq. (2)):
 *
 *       B[x] = sum over taps o of  C^g[o + r] * A[x + o]
 *
 *   Box shape: every offset o in [-r, r]^d.  Star shape: the offsets with at
 *   most one nonzero component (2rd + 1 taps, Section 3.4).  Taps are visited
 *   in lexicographic order of (o0, o1[, o2]); every multiply and add is a
 *   separate IEEE double operation (built with -ffp-contract=off).
 *
 *   Boundary (the paper states none; see the readings in the design notes):
 *     ZERO     - every grid point is updated; values outside the grid are 0.
 *     PERIODIC - indices wrap modulo the grid extent (non-negative modulo).
 *
 * Storage is C order, rightmost index contiguous (Section 4.1 footnote):
 * (i, j) in 2D and (i, j, k) in 3D.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_SHAPE_STAR 0
#define ORACLE_SHAPE_BOX 1
#define ORACLE_BC_ZERO 0
#define ORACLE_BC_PERIODIC 1

/* Non-negative remainder of v modulo n (n >= 1). */
static int64_t wrap_index(int64_t v, int64_t n) {
    int64_t m = v % n;
    if (m < 0) m += n;
    return m;
}

/* Whether tap offset o (ndim components) belongs to the shape. */
static int tap_in_shape(int ndim, int shape, const int* o) {
    if (shape == ORACLE_SHAPE_BOX) return 1;
    int nonzero = 0;
    for (int d = 0; d < ndim; ++d)
        if (o[d] != 0) nonzero++;
    return nonzero <= 1;
}

/* Value of A at position x + o under the boundary rule.  Returns 0.0 for a
 * zero-halo point outside the grid. */
static double fetch(int ndim, const int64_t* dims, int bc, const double* a,
                    const int64_t* x, const int* o) {
    int64_t flat = 0;
    for (int d = 0; d < ndim; ++d) {
        int64_t y = x[d] + (int64_t)o[d];
        if (bc == ORACLE_BC_PERIODIC) {
            y = wrap_index(y, dims[d]);
        } else if (y < 0 || y >= dims[d]) {
            return 0.0;
        }
        flat = flat * dims[d] + y;
    }
    return a[flat];
}

/* One Jacobi step B = S(A).  Returns 0 on success, -1 on bad arguments. */
int oracle_step(int ndim, const int64_t* dims, int radius, int shape, int bc,
                const double* coeffs, const double* a, double* b) {
    if (ndim < 2 || ndim > 3 || radius < 0 || !dims || !coeffs || !a || !b) return -1;
    for (int d = 0; d < ndim; ++d)
        if (dims[d] < 1) return -1;
    const int width = 2 * radius + 1;

    /* List the taps once, in lexicographic order of the offsets. */
    int ntaps_max = 1;
    for (int d = 0; d < ndim; ++d) ntaps_max *= width;
    int* taps = (int*)malloc(sizeof(int) * 3 * (size_t)ntaps_max);
    double* weights = (double*)malloc(sizeof(double) * (size_t)ntaps_max);
    if (!taps || !weights) {
        free(taps);
        free(weights);
        return -1;
    }
    int ntaps = 0;
    for (int t = 0; t < ntaps_max; ++t) {
        int o[3] = {0, 0, 0};
        int rem = t;
        int cidx = 0;
        for (int d = ndim - 1; d >= 0; --d) {
            o[d] = rem % width - radius;
            rem /= width;
        }
        /* C^g is indexed by o + r in C order. */
        for (int d = 0; d < ndim; ++d) cidx = cidx * width + (o[d] + radius);
        if (!tap_in_shape(ndim, shape, o)) continue;
        taps[3 * ntaps + 0] = o[0];
        taps[3 * ntaps + 1] = o[1];
        taps[3 * ntaps + 2] = o[2];
        weights[ntaps] = coeffs[cidx];
        ntaps++;
    }

    const int64_t n0 = dims[0];
    int64_t inner = 1;
    for (int d = 1; d < ndim; ++d) inner *= dims[d];

#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < n0; ++i0) {
        for (int64_t rest = 0; rest < inner; ++rest) {
            int64_t x[3];
            x[0] = i0;
            if (ndim == 2) {
                x[1] = rest;
            } else {
                x[1] = rest / dims[2];
                x[2] = rest % dims[2];
            }
            double s = 0.0;
            for (int t = 0; t < ntaps; ++t) {
                double v = fetch(ndim, dims, bc, a, x, &taps[3 * t]);
                double p = weights[t] * v;
                s = s + p;
            }
            b[i0 * inner + rest] = s;
        }
    }
    free(taps);
    free(weights);
    return 0;
}

/* `steps` Jacobi steps starting from a0; the final state is written to out.
 * steps == 0 copies a0.  Returns 0 on success, -1 on bad arguments or
 * allocation failure. */
int oracle_run(int ndim, const int64_t* dims, int radius, int shape, int bc,
               const double* coeffs, const double* a0, double* out, int64_t steps) {
    if (ndim < 2 || ndim > 3 || !dims || !a0 || !out || steps < 0) return -1;
    int64_t n = 1;
    for (int d = 0; d < ndim; ++d) {
        if (dims[d] < 1) return -1;
        n *= dims[d];
    }
    double* cur = (double*)malloc(sizeof(double) * (size_t)n);
    double* nxt = (double*)malloc(sizeof(double) * (size_t)n);
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return -1;
    }
    memcpy(cur, a0, sizeof(double) * (size_t)n);
    for (int64_t t = 0; t < steps; ++t) {
        int rc = oracle_step(ndim, dims, radius, shape, bc, coeffs, cur, nxt);
        if (rc != 0) {
            free(cur);
            free(nxt);
            return rc;
        }
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    memcpy(out, cur, sizeof(double) * (size_t)n);
    free(cur);
    free(nxt);
    return 0;
}

/* Thread control for timing runs: sets the OpenMP team size (n >= 1) and
 * returns the size that will be used. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
