/*
 * tdt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for what the GPU path
 * computes: X = T^{-1} F for the Toeplitz tridiagonal matrix
 *     T = tridiag{t_-1, t_0, t_1}          (paper, eq. (1); t_1 on the
 *                                            super-diagonal, t_-1 below)
 * and the adjoint of that map.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library; the product never does.
 * It shares no code, header or constant with the HIP path.
 *
 * Why the definition is the oracle: the dichotomy method is a direct solver.
 * Sec. 2.2 states that, once the end components of every sub-vector are known,
 * the remaining systems are solved "by any sequential version of the Thomas
 * algorithm", and the abstract and Sec. 4 claim accuracy comparable with the
 * sequential Thomas method.  In exact arithmetic the method reaches exactly
 * T^{-1} F, so the oracle is plain Gaussian elimination without pivoting on
 * the tridiagonal matrix (the Thomas algorithm), written out below:
 *
 *   forward:  u_1 = t0,            c'_1 = t1 / u_1,   d'_1 = f_1 / u_1
 *             u_i = t0 - t-1 c'_{i-1},  c'_i = t1 / u_i,
 *             d'_i = (f_i - t-1 d'_{i-1}) / u_i                 (i = 2..N)
 *   backward: x_N = d'_N,   x_i = d'_i - c'_i x_{i+1}           (i = N-1..1)
 *
 * A zero pivot u_i is reported as singular (status 1).
 *
 * Built with  gcc -O2 -ffp-contract=off -fopenmp  so that every product and
 * sum is rounded as written.  The long double variant (x87 extended, unit
 * roundoff 2^-64, forward error ~ cond(T) 2^-64) serves as "truth" for the
 * ill-conditioned systems, where the double result itself errs by
 * ~ cond(T) 2^-53.
 *
 * Quasi-Toeplitz matrices (paper, eq. (21)): the same matrix with t0+psi as
 * its first and t0+chi as its last diagonal entry (both added to the single
 * entry when N = 1).  The recurrence above is unchanged but for the pivot of
 * those rows: u_1 = t0 + psi, and t0 + chi in place of t0 in u_N.
 *
 * Adjoint (the differentiation extension): for L = <W, X> with X = T^{-1} F,
 *   gF = T^{-T} gX,  i.e. the same Thomas recurrence on T^T = tridiag{t1,t0,t-1}
 *   dL/dt0  = - sum_i   gF_i x_i
 *   dL/dt1  = - sum_i   gF_i x_{i+1}      (entries T_{i,i+1})
 *   dL/dt-1 = - sum_i   gF_{i+1} x_i      (entries T_{i+1,i})
 *   dL/dpsi = - gF_1 x_1,   dL/dchi = - gF_N x_N   (quasi-Toeplitz)
 * which follows from dX = -T^{-1} dT X.  The transposed solve is the paper's
 * remark in Sec. 2.3 that (A^T)^{-1} = (A^{-1})^T.  Sums are accumulated in
 * long double over all entries and right-hand sides.
 *
 * General tridiagonal matrices (the series of eq. (2) with a matrix whose
 * entries vary by row; the preliminary step of Sec. 2.3 is written for any
 * such A): row i reads a_i x_{i-1} + b_i x_i + c_i x_{i+1} = f_i, with a_1 and
 * c_N unused.  The recurrence is the one above with each row's own entries:
 *   u_1 = b_1,  u_i = b_i - a_i c'_{i-1},  c'_i = c_i / u_i,
 *   d'_i = (f_i - a_i d'_{i-1}) / u_i,  x_i = d'_i - c'_i x_{i+1}.
 * Its adjoint is the same solve with A^T (sub-diagonal c_{i-1}, super-diagonal
 * a_{i+1}) and the entry gradients, summed over the right-hand sides,
 *   dL/da_i = - sum gF_i x_{i-1},  dL/db_i = - sum gF_i x_i,
 *   dL/dc_i = - sum gF_i x_{i+1}   (0 for the unused a_1 and c_N).
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- one system, one right-hand side, double ---------------------------- */
/* diagonal entry of row i (0-based) of the quasi-Toeplitz matrix */
static double diag_f64(double t0, double psi, double chi, int64_t i, int64_t n)
{
    double d = t0;
    if (i == 0) d += psi;
    if (i == n - 1) d += chi;
    return d;
}

static int thomas_f64(double tm1, double t0, double t1, double psi, double chi, int64_t n,
                      const double *f, double *x, double *cp /* scratch n */)
{
    double u = diag_f64(t0, psi, chi, 0, n);
    if (u == 0.0) return 1;
    cp[0] = t1 / u;
    x[0] = f[0] / u;                       /* x holds d' until back-substitution */
    for (int64_t i = 1; i < n; ++i) {
        u = diag_f64(t0, psi, chi, i, n) - tm1 * cp[i - 1];
        if (u == 0.0) return 1;
        cp[i] = t1 / u;
        x[i] = (f[i] - tm1 * x[i - 1]) / u;
    }
    for (int64_t i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
    return 0;
}

/* ---- one system, one right-hand side, long double ------------------------ */
static long double diag_ld(long double t0, long double psi, long double chi, int64_t i,
                           int64_t n)
{
    long double d = t0;
    if (i == 0) d += psi;
    if (i == n - 1) d += chi;
    return d;
}

static int thomas_ld(long double tm1, long double t0, long double t1, long double psi,
                     long double chi, int64_t n, const long double *f, long double *x,
                     long double *cp)
{
    long double u = diag_ld(t0, psi, chi, 0, n);
    if (u == 0.0L) return 1;
    cp[0] = t1 / u;
    x[0] = f[0] / u;
    for (int64_t i = 1; i < n; ++i) {
        u = diag_ld(t0, psi, chi, i, n) - tm1 * cp[i - 1];
        if (u == 0.0L) return 1;
        cp[i] = t1 / u;
        x[i] = (f[i] - tm1 * x[i - 1]) / u;
    }
    for (int64_t i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
    return 0;
}

/* Long double variant: the same recurrence with every operation in x87
 * extended precision, rounded to double at the end.  work: 3*n long doubles. */
static int thomas_ld_to_f64(double tm1, double t0, double t1, double psi, double chi,
                            int64_t n, const double *f, double *xout, long double *work)
{
    long double *fl = work, *x = work + n, *cp = work + 2 * n;
    for (int64_t i = 0; i < n; ++i) fl[i] = (long double)f[i];
    int st = thomas_ld(tm1, t0, t1, psi, chi, n, fl, x, cp);
    if (st) return st;
    for (int64_t i = 0; i < n; ++i) xout[i] = (double)x[i];
    return 0;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* F, X: [M][N] row-major (one right-hand side per row).  psi, chi: corner
 * terms of eq. (21) (0 for a Toeplitz matrix).  precision: 0 = double,
 * 1 = long double.  Returns 0, 1 if some pivot is zero, 2 on allocation
 * failure, 3 on bad arguments.  nthreads <= 0 keeps the default. */
int oracle_solve(double tm1, double t0, double t1, double psi, double chi, int64_t N, int64_t M,
                 const double *F, double *X, int precision, int nthreads)
{
    if (N < 1 || M < 1 || !F || !X) return 3;
    set_threads(nthreads);
    int status = 0;
#pragma omp parallel
    {
        double *cp = (double *)malloc((size_t)N * sizeof(double));
        long double *wl = precision == 1
            ? (long double *)malloc((size_t)(3 * N) * sizeof(long double)) : NULL;
        int local = (cp && (precision != 1 || wl)) ? 0 : 2;
#pragma omp for schedule(static)
        for (int64_t m = 0; m < M; ++m) {
            if (local == 2) continue;
            int st = precision == 1
                ? thomas_ld_to_f64(tm1, t0, t1, psi, chi, N, F + m * N, X + m * N, wl)
                : thomas_f64(tm1, t0, t1, psi, chi, N, F + m * N, X + m * N, cp);
            if (st > local) local = st;
        }
#pragma omp critical
        { if (local > status) status = local; }
        free(cp); free(wl);
    }
    return status;
}

/* S systems packed back to back: system s occupies [offsets[s], offsets[s+1])
 * of F and X and has its own (tm1[s], t0[s], t1[s]) and corner terms
 * (psi[s], chi[s]; both arrays may be NULL for Toeplitz systems).  Systems are
 * handed out largest first with dynamic scheduling. */
int oracle_solve_varlen(int64_t S, const int64_t *offsets, const double *tm1,
                        const double *t0, const double *t1, const double *psi,
                        const double *chi, const double *F, double *X, int precision,
                        int nthreads)
{
    if (S < 1 || !offsets || !F || !X) return 3;
    int64_t nmax = 0;
    for (int64_t s = 0; s < S; ++s) {
        int64_t n = offsets[s + 1] - offsets[s];
        if (n < 1) return 3;
        if (n > nmax) nmax = n;
    }
    /* order by length, descending (simple insertion of indices) */
    int64_t *order = (int64_t *)malloc((size_t)S * sizeof(int64_t));
    if (!order) return 2;
    for (int64_t s = 0; s < S; ++s) order[s] = s;
    for (int64_t i = 1; i < S; ++i) {
        int64_t k = order[i], nk = offsets[k + 1] - offsets[k], j = i - 1;
        while (j >= 0 && offsets[order[j] + 1] - offsets[order[j]] < nk) {
            order[j + 1] = order[j]; --j;
        }
        order[j + 1] = k;
    }
    set_threads(nthreads);
    int status = 0;
#pragma omp parallel
    {
        double *cp = (double *)malloc((size_t)nmax * sizeof(double));
        long double *wl = precision == 1
            ? (long double *)malloc((size_t)(3 * nmax) * sizeof(long double)) : NULL;
        int local = (cp && (precision != 1 || wl)) ? 0 : 2;
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < S; ++i) {
            if (local == 2) continue;
            int64_t s = order[i], o = offsets[s], n = offsets[s + 1] - o;
            const double ps = psi ? psi[s] : 0.0, ch = chi ? chi[s] : 0.0;
            int st = precision == 1
                ? thomas_ld_to_f64(tm1[s], t0[s], t1[s], ps, ch, n, F + o, X + o, wl)
                : thomas_f64(tm1[s], t0[s], t1[s], ps, ch, n, F + o, X + o, cp);
            if (st > local) local = st;
        }
#pragma omp critical
        { if (local > status) status = local; }
        free(cp); free(wl);
    }
    free(order);
    return status;
}

/* Adjoint of X = T^{-1} F for M right-hand sides sharing one T.
 * gX, X: [M][N] in; gF: [M][N] out; gt[5] = (dL/dt-1, dL/dt0, dL/dt1,
 * dL/dpsi, dL/dchi) summed over all right-hand sides. */
int oracle_adjoint(double tm1, double t0, double t1, double psi, double chi, int64_t N,
                   int64_t M, const double *gX, const double *X, double *gF, double *gt,
                   int nthreads)
{
    if (N < 1 || M < 1 || !gX || !X || !gF || !gt) return 3;
    /* gF = T^{-T} gX: Thomas on the transpose, i.e. t1 and t-1 exchanged
       (the corner terms sit on the diagonal and stay) */
    int st = oracle_solve(t1, t0, tm1, psi, chi, N, M, gX, gF, 0, nthreads);
    if (st) return st;
    long double s_m1 = 0.0L, s_0 = 0.0L, s_p1 = 0.0L, s_ps = 0.0L, s_ch = 0.0L;
    for (int64_t m = 0; m < M; ++m) {
        const double *g = gF + m * N, *x = X + m * N;
        for (int64_t i = 0; i < N; ++i) {
            s_0 += (long double)g[i] * x[i];
            if (i + 1 < N) {
                s_p1 += (long double)g[i] * x[i + 1];
                s_m1 += (long double)g[i + 1] * x[i];
            }
        }
        s_ps += (long double)g[0] * x[0];
        s_ch += (long double)g[N - 1] * x[N - 1];
    }
    gt[0] = (double)(-s_m1);
    gt[1] = (double)(-s_0);
    gt[2] = (double)(-s_p1);
    gt[3] = (double)(-s_ps);
    gt[4] = (double)(-s_ch);
    return 0;
}

/* Varlen adjoint: per system (dL/dt-1, dL/dt0, dL/dt1, dL/dpsi, dL/dchi),
 * gt: [S][5]; psi, chi as in oracle_solve_varlen. */
int oracle_adjoint_varlen(int64_t S, const int64_t *offsets, const double *tm1,
                          const double *t0, const double *t1, const double *psi,
                          const double *chi, const double *gX, const double *X, double *gF,
                          double *gt, int nthreads)
{
    if (S < 1 || !offsets || !gX || !X || !gF || !gt) return 3;
    int st = oracle_solve_varlen(S, offsets, t1, t0, tm1, psi, chi, gX, gF, 0, nthreads);
    if (st) return st;
    for (int64_t s = 0; s < S; ++s) {
        int64_t o = offsets[s], n = offsets[s + 1] - o;
        const double *g = gF + o, *x = X + o;
        long double s_m1 = 0.0L, s_0 = 0.0L, s_p1 = 0.0L;
        for (int64_t i = 0; i < n; ++i) {
            s_0 += (long double)g[i] * x[i];
            if (i + 1 < n) {
                s_p1 += (long double)g[i] * x[i + 1];
                s_m1 += (long double)g[i + 1] * x[i];
            }
        }
        gt[5 * s + 0] = (double)(-s_m1);
        gt[5 * s + 1] = (double)(-s_0);
        gt[5 * s + 2] = (double)(-s_p1);
        gt[5 * s + 3] = (double)(-((long double)g[0] * x[0]));
        gt[5 * s + 4] = (double)(-((long double)g[n - 1] * x[n - 1]));
    }
    return 0;
}

/* ---- general tridiagonal matrix -------------------------------------------- */
static int thomas_gen_f64(const double *a, const double *b, const double *c, int64_t n,
                          const double *f, double *x, double *cp)
{
    double u = b[0];
    if (u == 0.0) return 1;
    cp[0] = c[0] / u;
    x[0] = f[0] / u;
    for (int64_t i = 1; i < n; ++i) {
        u = b[i] - a[i] * cp[i - 1];
        if (u == 0.0) return 1;
        cp[i] = c[i] / u;
        x[i] = (f[i] - a[i] * x[i - 1]) / u;
    }
    for (int64_t i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
    return 0;
}

/* the same in long double, rounded to double at the end; work: 2*n */
static int thomas_gen_ld(const double *a, const double *b, const double *c, int64_t n,
                         const double *f, double *xout, long double *work)
{
    long double *x = work, *cp = work + n;
    long double u = (long double)b[0];
    if (u == 0.0L) return 1;
    cp[0] = (long double)c[0] / u;
    x[0] = (long double)f[0] / u;
    for (int64_t i = 1; i < n; ++i) {
        u = (long double)b[i] - (long double)a[i] * cp[i - 1];
        if (u == 0.0L) return 1;
        cp[i] = (long double)c[i] / u;
        x[i] = ((long double)f[i] - (long double)a[i] * x[i - 1]) / u;
    }
    for (int64_t i = n - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
    for (int64_t i = 0; i < n; ++i) xout[i] = (double)x[i];
    return 0;
}

/* X = A^{-1} F for M right-hand sides ([M][N]) sharing the general matrix
 * with rows (a_i, b_i, c_i); precision and status as oracle_solve. */
int oracle_solve_general(const double *a, const double *b, const double *c, int64_t N,
                         int64_t M, const double *F, double *X, int precision, int nthreads)
{
    if (N < 1 || M < 1 || !a || !b || !c || !F || !X || (precision != 0 && precision != 1))
        return 3;
    set_threads(nthreads);
    int status = 0;
#pragma omp parallel
    {
        void *work = precision == 1 ? malloc((size_t)(2 * N) * sizeof(long double))
                                    : malloc((size_t)N * sizeof(double));
        int local = work ? 0 : 2;
#pragma omp for schedule(static)
        for (int64_t m = 0; m < M; ++m) {
            if (local == 2) continue;
            int st = precision == 1
                ? thomas_gen_ld(a, b, c, N, F + m * N, X + m * N, (long double *)work)
                : thomas_gen_f64(a, b, c, N, F + m * N, X + m * N, (double *)work);
            if (st > local) local = st;
        }
#pragma omp critical
        { if (local > status) status = local; }
        free(work);
    }
    return status;
}

/* Adjoint for the general matrix: gF = A^{-T} gX ([M][N]) and the entry
 * gradients ga, gb, gc ([N] each) summed over the right-hand sides. */
int oracle_adjoint_general(const double *a, const double *b, const double *c, int64_t N,
                           int64_t M, const double *gX, const double *X, double *gF,
                           double *ga, double *gb, double *gc, int nthreads)
{
    if (N < 1 || M < 1 || !a || !b || !c || !gX || !X || !gF || !ga || !gb || !gc) return 3;
    double *at = malloc((size_t)N * sizeof(double)), *ct = malloc((size_t)N * sizeof(double));
    if (!at || !ct) {
        free(at);
        free(ct);
        return 2;
    }
    /* A^T: row i has c_{i-1} left of the diagonal and a_{i+1} right of it */
    for (int64_t i = 0; i < N; ++i) {
        at[i] = i > 0 ? c[i - 1] : 0.0;
        ct[i] = i + 1 < N ? a[i + 1] : 0.0;
    }
    int st = oracle_solve_general(at, b, ct, N, M, gX, gF, 0, nthreads);
    free(at);
    free(ct);
    if (st) return st;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        long double sa = 0.0L, sb = 0.0L, sc = 0.0L;
        for (int64_t m = 0; m < M; ++m) {
            const double *g = gF + m * N, *x = X + m * N;
            sb += (long double)g[i] * x[i];
            if (i > 0) sa += (long double)g[i] * x[i - 1];
            if (i + 1 < N) sc += (long double)g[i] * x[i + 1];
        }
        ga[i] = (double)(-sa);
        gb[i] = (double)(-sb);
        gc[i] = (double)(-sc);
    }
    return 0;
}

/* Threads the OpenMP runtime would use after set_threads(nthreads). */
int oracle_threads(int nthreads) { return set_threads(nthreads); }
