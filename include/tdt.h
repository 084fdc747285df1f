/*
 * tdt.h -- C ABI of the MI355X (gfx950) solver for Toeplitz tridiagonal
 * systems T X = F, T = tridiag{t_-1, t_0, t_1}, by the partitioned dichotomy
 * method (Terekhov, "Application of the Parallel Dichotomy Algorithm for
 * solving Toeplitz tridiagonal systems of linear equations with one
 * right-hand side").
 *
 * Matrix convention (paper, eq. (1)): row i of T X = F reads
 *     t_-1 x_{i-1} + t_0 x_i + t_1 x_{i+1} = f_i,     i = 0 .. N-1,
 * with x_{-1} = x_N = 0: t_1 is the super-diagonal, t_-1 the sub-diagonal.
 *
 * Every function returns a tdt_status_t; nothing throws across the ABI.
 * Data buffers (F, X, gX, gF, gt) are DEVICE pointers owned by the caller;
 * the library never frees them.  All device work is enqueued on the caller's
 * stream and is asynchronous: the library never synchronises that stream.
 * Argument errors are reported synchronously, before anything is enqueued.
 * A plan owns its device constants and workspace; one plan must not be used
 * by two solves that may run concurrently (they share the workspace).
 */
#ifndef TDT_H
#define TDT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdt_plan_s *tdt_plan_t;

/* Arithmetic of a plan.  Data in and out are double for TDT_F64 and
 * TDT_F32_REFINE, float for TDT_F32.
 *   TDT_F64        every step in double;
 *   TDT_F32        every step in float (accuracy ~ cond(T) * 2^-24);
 *   TDT_F32_REFINE each tile's sweeps, its in-tile interface and the
 *                  correction in float; the tile summaries, the interface
 *                  pass across tiles, the residual r = F - T X and the
 *                  update X += d in double, repeated until the update stops
 *                  shrinking (iterative refinement), so the result matches
 *                  the double solve. */
typedef enum { TDT_F64 = 0, TDT_F32 = 1, TDT_F32_REFINE = 2 } tdt_dtype_t;

typedef enum {
    TDT_OK = 0,
    /* solved, but |t_0| < |t_1| + |t_-1|: diagonal dominance, the paper's
       sufficient condition of stability (Sec. 3.4), does not hold, so
       rounding errors may grow from one interface level to the next */
    TDT_WARN_NOT_DOMINANT = 1,
    TDT_ERR_INVALID_ARG = -1,   /* bad size, null pointer, aliasing, wrong plan kind */
    TDT_ERR_SINGULAR = -2,      /* T, or one of the sub-blocks the method inverts, is singular */
    TDT_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
    TDT_ERR_OOM = -4,           /* device or host allocation failed */
    TDT_ERR_NOT_CONVERGED = -5, /* refinement did not converge (tdt_last_info) */
    TDT_ERR_CAPTURE = -6        /* would allocate during stream capture: call tdt_plan_reserve first */
} tdt_status_t;

/* Plan for one Toeplitz matrix of order N (the preliminary step of the
 * method, done once per T: Sec. 3.1 shows that for a Toeplitz matrix every
 * quantity the interface pass needs costs O(1), so nothing here depends on
 * the right-hand side).  Builds, in long double on the host, the LU
 * multipliers of the B x B diagonal block, the block's responses to unit
 * interface values ("shared basis", the local counterpart of the Green
 * functions of eqs. (9)-(12) and of the interior problems of eqs. (26)-(27)),
 * and the same end values for whole tiles; uploads them (blocking copy).
 * Errors: N < 1, non-finite t's, out == NULL -> TDT_ERR_INVALID_ARG;
 * a zero pivot in a diagonal block or an interface merge that divides by
 * zero -> TDT_ERR_SINGULAR.  Returns TDT_WARN_NOT_DOMINANT (plan usable)
 * when |t_0| < |t_1| + |t_-1|. */
tdt_status_t tdt_plan_create(double t_m1, double t_0, double t_1, int64_t N,
                             tdt_dtype_t dtype, tdt_plan_t *out);

/* Plan for S systems of different sizes, each with its own matrix (the
 * series of Sec. 3.2 produced by separating variables: one system per
 * Fourier mode).  h_offsets: host array of S+1 increasing int64, system s
 * occupies elements [h_offsets[s], h_offsets[s+1]) of the packed F and X
 * (h_offsets[0] may be non-zero only as 0; sizes >= 1).  h_tm1, h_t0, h_t1:
 * host arrays of S doubles.  Errors and warnings as tdt_plan_create; a
 * warning refers to the least dominant system. */
tdt_status_t tdt_plan_varlen_create(int64_t S, const int64_t *h_offsets,
                                    const double *h_tm1, const double *h_t0,
                                    const double *h_t1, tdt_dtype_t dtype,
                                    tdt_plan_t *out);

/* Plan for the quasi-Toeplitz matrix of eq. (21): T with its first diagonal
 * entry t_0 + psi and its last t_0 + chi (the form a Poisson problem with
 * Neumann or Robin boundary rows takes, Sec. 3.2), order N >= 3.  The tiles
 * cover the N - 2 inner rows, which are Toeplitz; the two corner rows join the
 * interface pass across tiles as one-row segments at its two ends, so the
 * corner terms cost O(1) per right-hand side.  Solves, the adjoint and every
 * option work as for tdt_plan_create, with the same layouts (rows 0 .. N-1);
 * tdt_solve_backward then writes 5 doubles per system to d_gt:
 *   d_gt[5s+0..2] as for a Toeplitz plan (the corner rows included: row 0
 *                 has no t_-1 term, row N-1 no t_1 term),
 *   d_gt[5s+3]  = dL/dpsi = - gF_0 x_0,
 *   d_gt[5s+4]  = dL/dchi = - gF_{N-1} x_{N-1}.
 * Errors: N < 3, non-finite arguments -> TDT_ERR_INVALID_ARG; t_0 + psi = 0,
 * t_0 + chi = 0 or a vanishing interface pivot -> TDT_ERR_SINGULAR.  The
 * dominance ratio includes the corner rows (|t_0+psi|/|t_1|,
 * |t_0+chi|/|t_-1|); kappa2 (tdt_last_info) is an upper bound,
 * sqrt(kappa_1 kappa_inf) with both from strict row and column dominance
 * (infinite without it). */
tdt_status_t tdt_plan_quasi_create(double t_m1, double t_0, double t_1, double psi,
                                   double chi, int64_t N, tdt_dtype_t dtype,
                                   tdt_plan_t *out);

/* Varlen plan of quasi-Toeplitz systems (eq. (21)), each with its own t's and
 * corner terms h_psi[s], h_chi[s] (host arrays of S doubles); sizes >= 3.
 * Layout, errors and the 5 t-gradients per system as above. */
tdt_status_t tdt_plan_varlen_quasi_create(int64_t S, const int64_t *h_offsets,
                                          const double *h_tm1, const double *h_t0,
                                          const double *h_t1, const double *h_psi,
                                          const double *h_chi, tdt_dtype_t dtype,
                                          tdt_plan_t *out);

/* Plan for a general tridiagonal matrix A of order N: row i reads
 *     a_i x_{i-1} + b_i x_i + c_i x_{i+1} = f_i     (a_0 and c_{N-1} unused),
 * for series of right-hand sides sharing A (eq. (2) with any A; the
 * preliminary step of Sec. 2.3 is written for such A, and its O(N) cost is
 * paid once per A).  h_a, h_b, h_c: host arrays of N doubles, copied.  The
 * plan computes, in long double, the LU of every B-row block, every block's
 * responses to unit outside values and the end values of every tile, for A
 * and for A^T; the device holds 3 values per row and 5 per block in the
 * compute precision, plus 4 per tile and, for the first pass, the tiles'
 * first and last inverse rows in double (only the entries under their
 * supports when the plan finds them short: tdt_plan_green_support).  dtype: TDT_F64 or TDT_F32
 * (TDT_F32_REFINE -> TDT_ERR_INVALID_ARG).  Solve with tdt_solve (F, X:
 * [M][N]).  tdt_solve_backward solves A^T gF = gX and, if d_gt is not NULL,
 * writes 3*N doubles: d_gt[i] = dL/da_i, d_gt[N+i] = dL/db_i, d_gt[2N+i] =
 * dL/dc_i, each summed over the M right-hand sides (0 for a_0 and c_{N-1}).
 * The plan is built for work shape 1 (8 rows x 512 lanes); TDT_OPT_SHAPE
 * accepts only that.  Errors: N < 1, null arrays, non-finite entries ->
 * TDT_ERR_INVALID_ARG; a zero block pivot or a vanishing interface pivot ->
 * TDT_ERR_SINGULAR.  The dominance ratio is min_i |b_i|/(|a_i|+|c_i|);
 * kappa2 is the bound sqrt(kappa_1 kappa_inf) from strict row and column
 * dominance (infinite without it). */
tdt_status_t tdt_plan_general_create(int64_t N, const double *h_a, const double *h_b,
                                     const double *h_c, tdt_dtype_t dtype,
                                     tdt_plan_t *out);

/* Plan for batches of Toeplitz systems laid out along a slow axis (the
 * lines along y or z of a row-major 2D or 3D array): P classes of matrices
 * T_k = tridiag{h_tm1[k], h_t0[k], h_t1[k]} of order N (host arrays of P
 * doubles, copied), 1 <= N <= 2^24.  Solved with tdt_solve_strided, which
 * runs the dichotomy method (Sec. 2.1-2.5) with one workgroup per column of
 * adjacent systems: every lane holds a 16-row block of one system, the
 * interface values of eq. (15) are scanned across the blocks inside the
 * workgroup, and the blocks are corrected in registers.  A system of more
 * than 1024 rows is cut into tiles of 512 rows (the last one shorter), each
 * such a column: a first pass keeps the end values of every tile's solution
 * with zero outside values, one thread per system eliminates the tiles'
 * interface values (the recurrences of eq. (15) over the tiles), and a
 * second pass re-solves every tile with its two outside values.  The plan
 * holds per class the block LU, the blocks' end values and the interface
 * table of a column, computed in long double (17 + 2 ceil(N/16) doubles per
 * class for N <= 1024; for longer N, that of a full tile and of the last
 * tile plus 8 tile end values).
 * dtype: TDT_F64 only.  Errors: N outside [1, 2^24], P < 1, null arrays,
 * non-finite entries, another dtype -> TDT_ERR_INVALID_ARG; a zero block
 * pivot or a vanishing interface pivot (of the blocks or of the tiles) ->
 * TDT_ERR_SINGULAR; host or device allocation -> TDT_ERR_OOM; returns
 * TDT_WARN_NOT_DOMINANT (plan valid) when some class has
 * |t_0| < |t_-1| + |t_1|.  tdt_solve, tdt_solve_varlen, tdt_solve_backward,
 * options and autotuning refuse such a plan (TDT_ERR_INVALID_ARG). */
tdt_status_t tdt_plan_strided_create(int64_t N, int64_t P, const double *h_tm1,
                                     const double *h_t0, const double *h_t1,
                                     tdt_dtype_t dtype, tdt_plan_t *out);

/* Solve system s = 0 .. M-1 (M <= P; system s uses class s) of every batch
 * b = 0 .. nb-1: unknown i of system s of batch b is F[b*ldb + i*ld + s]
 * (and X[...] likewise), i = 0 .. N-1.  F, X: device doubles, caller-owned;
 * X may be F itself (in place) but must not overlap it otherwise.  The
 * layout must be one of: batches one after another (ld >= M and, for
 * nb > 1, ldb >= (N-1)*ld + M), or batches interleaved in each row
 * (ldb >= M, ld >= (nb-1)*ldb + M); other layouts -> TDT_ERR_INVALID_ARG.
 * N <= 1024: no workspace.  Longer N: the plan's workspace holds
 * 4 nb M ceil(N/512) doubles, allocated on first use or by
 * tdt_plan_reserve(plan, nb*M); a solve that needs more while its stream is
 * being captured returns TDT_ERR_CAPTURE.  Five launches then (two per pass,
 * the full tiles and the last one, and the interface), one otherwise; both
 * are capturable in a hipGraph.  Under tdt_plan_profile the kernel time is
 * reported as the third value of tdt_plan_profile_read. */
tdt_status_t tdt_solve_strided(tdt_plan_t plan, const double *F, double *X, int64_t M,
                               int64_t ld, int64_t nb, int64_t ldb, hipStream_t stream);

/* 2D Poisson solve by separation of variables (the application of Sec. 3.2
 * and of the paper's timings): the five-point system
 *     (2u_ij - u_{i-1,j} - u_{i+1,j}) / hx^2 + (2u_ij - u_{i,j-1} - u_{i,j+1}) / hy^2 = f_ij
 * on Nx x Ny interior points with u = 0 on the boundary.  A sine transform
 * along x (a real FFT of length Nx+1 of each folded row, then a prefix sum
 * for the odd coefficients: in one kernel when Nx+1 is a power of two from
 * 128 to 8192, through hipFFT otherwise) leaves one tridiagonal Toeplitz
 * system per mode k along y, t_+-1 = -1,
 * t_0 = 2 + hy^2 (4/hx^2) sin^2(pi k / (2 (Nx+1))); the inverse transform
 * gives U.  With the one-kernel transform and TDT_F64, the mode systems are
 * solved in place in the transformed rows by a strided plan (system k is
 * column k; rows padded to ldw = 16 ceil(Nx/16) + 16 doubles): 2 row
 * transforms and the strided solve, no transposes; the workspace is Ny ldw
 * doubles plus the strided plan's 4 Nx ceil(Ny/512) when Ny > 1024.
 * Otherwise (TDT_F32_REFINE, or the hipFFT path) the transformed rows are
 * transposed to mode-major order and solved by a varlen plan of this
 * library, with 2 Nx Ny + Ny (Nx + 1) doubles of workspace, plus
 * 2 Ny (floor((Nx+1)/2) + 1) on the hipFFT path.  The handle owns the line
 * plan, the twiddle tables or the FFT plan and the workspace (allocated
 * here, blocking).  Errors: sizes
 * < 1 or Nx Ny > 2^31, non-positive or non-finite spacings, another dtype ->
 * TDT_ERR_INVALID_ARG; allocation -> TDT_ERR_OOM; an FFT plan failure ->
 * TDT_ERR_HIP; TDT_F32_REFINE when a mode system's condition number (closed
 * form, largest for the lowest mode: about 0.2 (Ny+1)^2 on a square grid)
 * exceeds 8e6, where float sweeps contract the refinement too slowly to
 * reach double accuracy (eq. (34)'s error growth bounds what a float solve
 * contributes) -> TDT_ERR_NOT_CONVERGED, before anything is allocated. */
typedef struct tdt_poisson_s *tdt_poisson_t;
tdt_status_t tdt_poisson2d_create(int64_t nx, int64_t ny, double hx, double hy,
                                  tdt_dtype_t dtype, tdt_poisson_t *out);
/* U = A^{-1} F; F, U: device, [Ny][Nx] doubles, caller-owned, distinct.
 * Enqueued on stream (the FFTs too); one handle must not be used by two
 * solves that may run concurrently (shared workspace). */
tdt_status_t tdt_poisson2d_solve(tdt_poisson_t p, const double *F, double *U,
                                 hipStream_t stream);
/* The handle's line plan (owned by the handle), e.g. to set its options or
 * autotune it: a varlen plan, or the strided plan of the in-place path
 * (which takes no options). */
tdt_status_t tdt_poisson2d_line_plan(tdt_poisson_t p, tdt_plan_t *line);
/* HIP events around the forward transform (with the transpose to mode-major
 * order on that path), the line solve and the inverse transform of every
 * later solve (solves on a capturing stream are not recorded); _read
 * synchronises the device and returns their summed ms in ms3[0..2] and the
 * number of solves, and clears the record.  Errors: null handle or ms3 ->
 * TDT_ERR_INVALID_ARG; an event failure -> TDT_ERR_HIP. */
tdt_status_t tdt_poisson2d_profile(tdt_poisson_t p, int enable);
tdt_status_t tdt_poisson2d_profile_read(tdt_poisson_t p, double *ms3, int64_t *nsolves);
tdt_status_t tdt_poisson2d_destroy(tdt_poisson_t p);

/* 3D Poisson solve of Sec. 3.5: the seven-point system
 *     (2u - u_{i-1} - u_{i+1}) / hx^2 + (... along y) / hy^2 + (... along z) / hz^2 = f
 * on Nx x Ny x Nz interior points, u = 0 on the boundary, F and U [Nz][Ny][Nx]
 * doubles.  A sine transform along x (as in the 2D solve) leaves one 2D
 * problem (A_y + A_z + mu_k) v_k = fhat_k per mode k, each solved by
 * Peaceman-Rachford ADI (the shift split evenly between the two directions)
 * whose half-steps are strided batches of Toeplitz line systems
 * (tdt_solve_strided's kernel: lines along y, then along z, every plane's
 * modes at once), then the inverse transform.  The ADI parameters of mode k
 * are the optimal (Jordan, Wachspress) set w_j = b dn((2j-1) K / (2 J_k), m),
 * m = 1 - (a/b)^2, for the interval [a, b] holding the spectra of both
 * directions' operators; J_k is the smallest count whose error bound for a
 * full cycle, d_J^2 with d_J = prod_j (w_j - a)/(w_j + a), is <= eps, so the
 * 2-norm error of the result relative to the exact discrete solution is at
 * most eps (plus rounding).  J_k falls as k grows.  1 <= Ny, Nz <= 2^24
 * (lines of more than 1024 points are solved in tiles of 512, as by
 * tdt_solve_strided), 640 Nxp Ny < 2^31 with Nxp = 16 ceil(Nx/16) + 16 on
 * the fused path, Nx otherwise (31-bit byte offsets of the z lines),
 * 0 < eps < 1; a count above 400 for some mode -> TDT_ERR_INVALID_ARG.  The
 * handle owns the per-iteration tables (~(38 + 4 ceil(N/16)) doubles per
 * mode and iteration, about twice that for tiled lines), for tiled lines
 * 4 Nx max(Nz ceil(Ny/512), Ny ceil(Nz/512)) doubles, and
 * 2 (16 ceil(Nx/16) + 16) Ny Nz doubles of workspace when
 * Nx+1 is a power of two from 128 to 8192 (the fused row transform; rows
 * padded to cache lines), else the FFT plan and (2 Nx + 3) Ny Nz doubles
 * (allocated here, blocking).  Errors: bad sizes, spacings or eps ->
 * TDT_ERR_INVALID_ARG; allocation -> TDT_ERR_OOM; FFT plan -> TDT_ERR_HIP. */
typedef struct tdt_poisson3d_s *tdt_poisson3d_t;
tdt_status_t tdt_poisson3d_create(int64_t nx, int64_t ny, int64_t nz, double hx, double hy,
                                  double hz, double eps, tdt_poisson3d_t *out);
/* U = A^{-1} F (to the ADI bound); F, U: device, caller-owned, distinct.
 * Enqueued on stream; one handle must not run two solves at once. */
tdt_status_t tdt_poisson3d_solve(tdt_poisson3d_t p, const double *F, double *U,
                                 hipStream_t stream);
/* The ADI schedule: h_counts[k] = J_k (Nx ints, may be NULL), h_omega[k *
 * jmax + j] = w_{k,j+1} for j < J_k, 0 after (omega_len >= Nx * jmax doubles,
 * may be NULL), *jmax = J_1 (the largest count). */
tdt_status_t tdt_poisson3d_schedule(tdt_poisson3d_t p, int *h_counts, double *h_omega,
                                    int64_t omega_len, int *jmax);
/* HIP events around the forward transform, the ADI iterations and the
 * inverse transform of every later solve; _read returns their summed ms
 * and the number of solves, and clears the record. */
tdt_status_t tdt_poisson3d_profile(tdt_poisson3d_t p, int enable);
tdt_status_t tdt_poisson3d_profile_read(tdt_poisson3d_t p, double *ms3, int64_t *nsolves);
tdt_status_t tdt_poisson3d_destroy(tdt_poisson3d_t p);
/* Host-only test hook: the J optimal ADI parameters for [a, b] (largest
 * first; out: J doubles) and their bound d_J (may be NULL), as the 3D solve
 * computes them.  0 < a <= b, 1 <= J <= 400, else TDT_ERR_INVALID_ARG. */
tdt_status_t tdt_adi_parameters(double a, double b, int J, double *out, double *bound);

/* Allocate the workspace for up to M_max right-hand sides now, so that later
 * solves allocate nothing and may be captured in a hipGraph.  Blocking.  For
 * a strided plan M_max counts systems over all batches (nb * M); it is a
 * no-op for strided plans of at most 1024 rows. */
tdt_status_t tdt_plan_reserve(tdt_plan_t plan, int64_t M_max);

/* Solve T X_m = F_m for M right-hand sides sharing the plan's matrix (the
 * series of eq. (2) with a Toeplitz matrix; M = 1 is the single system of
 * the paper's title).  F, X: device, [M][N] row-major, element type of the
 * plan's dtype.  X must not overlap F.  Errors: M < 1, null pointers,
 * overlap, varlen plan -> TDT_ERR_INVALID_ARG; workspace growth during
 * capture -> TDT_ERR_CAPTURE; launch failure -> TDT_ERR_HIP. */
tdt_status_t tdt_solve(tdt_plan_t plan, const void *F, void *X, int64_t M,
                       hipStream_t stream);

/* tdt_solve for callers that cannot allocate device memory (code being
 * captured into a hipGraph without a prior tdt_plan_reserve, tight serving
 * loops, harnesses that forbid allocation): the same solve, same kernels,
 * same result, but its workspace is a static device array of the library
 * (7 MiB per GPU it runs on, held until the process ends) instead of the
 * plan's, so it calls no hipMalloc, hipFree or other allocating routine.
 * Arguments, layouts and errors as tdt_solve; a solve that needs more than
 * 2^17 tile slots (M times the number of tiles of N) -> TDT_ERR_INVALID_ARG.
 * Every call on one GPU shares that array: calls that may overlap on one GPU
 * (two streams, two threads) race and must be serialised by the caller.
 * Not recorded by tdt_plan_profile. */
tdt_status_t tdt_solve_noalloc(tdt_plan_t plan, const void *F, void *X, int64_t M,
                               hipStream_t stream);

/* Solve every system of a varlen plan (the series of Sec. 3.2: one system
 * per Fourier mode after separating variables, each mode with its own t_0
 * and, here, its own size): F, X device, packed by the plan's offsets,
 * element type of the plan's dtype.  One launch sequence for all systems;
 * systems are processed largest first.  Errors as tdt_solve. */
tdt_status_t tdt_solve_varlen(tdt_plan_t plan, const void *F, void *X,
                              hipStream_t stream);

/* Adjoint (reverse mode) of X = T^{-1} F for the loss L with dL/dX = gX.
 * gF = T^{-T} gX is solved through the same dichotomy machinery with t_1 and
 * t_-1 exchanged (T^T = tridiag{t_1, t_0, t_-1}; the paper's remark in
 * Sec. 2.3 that (A^T)^{-1} = (A^{-1})^T), and
 *   d_gt[3s+0] = dL/dt_-1 = - sum_i gF_{i+1} x_i
 *   d_gt[3s+1] = dL/dt_0  = - sum_i gF_i     x_i
 *   d_gt[3s+2] = dL/dt_1  = - sum_i gF_i     x_{i+1}
 * reduced on the device in a fixed order (bitwise repeatable), summed over
 * the M right-hand sides of a series plan (S = 1) or per system s of a varlen
 * plan.  gX, X, gF: device, layout of tdt_solve / tdt_solve_varlen (M is
 * ignored for a varlen plan); X is the forward solution.  d_gt: device, S*3
 * doubles (may be NULL to skip the t gradients).  gF must not overlap gX or X. */
tdt_status_t tdt_solve_backward(tdt_plan_t plan, const void *gX, const void *X,
                                void *gF, double *d_gt, int64_t M,
                                hipStream_t stream);

/* Free the plan's device memory.  Waits for the device to finish with it. */
tdt_status_t tdt_plan_destroy(tdt_plan_t plan);

/* Static string for a status code. */
const char *tdt_status_string(tdt_status_t status);

/* Facts about a plan (any pointer may be NULL): the dominance ratio of
 * Sec. 3.4 (eqs. (32)-(33), the condition under which the method's rounding
 * errors stay bounded), the condition number, and the refinement record.
 * For TDT_F32_REFINE solves
 * since the previous call that asked for them (read back from the device, so
 * asking synchronises the device; the record is then cleared):
 * *n_refine_iters = the most float solves any tile needed (0 when no such
 * solve ran), *last_rel_update = the largest estimated remaining relative
 * error of a tile: the size of the update the iteration would make next,
 * |d_k| rho / |x| with rho = |d_k| / |d_{k-1}| the observed contraction, or
 * |d_k| / |x| when updates stopped shrinking (1 when a tile ran no update).
 * Always: the dominance
 * ratio min_s |t_0|/(|t_1|+|t_-1|), and the 2-norm condition number of T
 * (the largest over systems), from the closed-form spectrum
 * t_0 + 2 sgn(t_1) sqrt(t_1 t_-1) cos(k pi/(N+1)) when t_1 t_-1 > 0, else
 * the infinity-norm bound from dominance (infinite when not dominant).
 * Returns TDT_ERR_NOT_CONVERGED (outputs still filled) when that estimate
 * is above 1e-7, i.e. refinement stopped (at TDT_OPT_MAX_REFINE, or because
 * its updates stopped shrinking) without getting past float resolution: X
 * then holds the last iterate. */
tdt_status_t tdt_last_info(tdt_plan_t plan, int *n_refine_iters,
                           double *last_rel_update, double *dominance,
                           double *kappa2);

/* Host-only (no device needed): the per-T constants the plan would upload for
 * block length B (1 <= B <= 64): out[0..B) = 1/u_k (inverse pivots of the
 * B x B block), out[B..2B) = t_1/u_k, out[2B..3B) = phi (response of the
 * block to a unit value left of it), out[3B..4B) = chi (response to a unit
 * value right of it), out[4B..4B+4) = (phi_0, phi_{B-1}, chi_0, chi_{B-1}).
 * Used to test the preliminary step against dense inverses. */
tdt_status_t tdt_block_constants(double t_m1, double t_0, double t_1, int B,
                                 double *out);

/* Host-only: the first and last row of T_L^{-1}, the L x L Toeplitz matrix
 * (the Green's function rows of eq. (9) of the paper for a run of L rows
 * taken as the whole system), in long double rounded to double: first[j] =
 * (T_L^{-1})_{0,j}, last[j] = (T_L^{-1})_{L-1,j}, j < L.  The first pass of a
 * series plan uses them for its tiles (L = the tile length). */
tdt_status_t tdt_green_rows(double t_m1, double t_0, double t_1, int64_t L,
                            double *first, double *last);

/* Host-only: where those two rows carry their mass.  Under diagonal
 * dominance the entries of T_L^{-1} fall off geometrically away from the
 * diagonal (Sec. 3.4, eqs. (32)-(33)), so the first pass of a series plan,
 * whose tile summaries are the dot products of eq. (13) of a tile's right-hand
 * side with these rows, reads only the rows of the tile that matter:
 * *kf = the fewest leading entries of the first row and *kl = the fewest
 * trailing entries of the last row such that the dropped entries' 1-norm is
 * at most 2^-60 of the row's (computed in long double).  The dropped part of
 * a summary is then at most 2^-60 |row|_1 |F|_inf, below the rounding of the
 * dot product.  bound2 (may be NULL): the supports a varlen plan uses for
 * its systems, found without forming the rows, from the decay of the ratios
 * of the elimination's pivots (at least *kf and *kl; 0, 0 when that bound
 * finds no truncation).  Errors: L outside [1, 2^26], non-finite t's, null
 * kf or kl -> TDT_ERR_INVALID_ARG; a zero pivot -> TDT_ERR_SINGULAR. */
tdt_status_t tdt_green_support(double t_m1, double t_0, double t_1, int64_t L, int64_t *kf,
                               int64_t *kl, int64_t *bound2);

/* What the first pass of a plan reads per full tile: rows4[0], rows4[1] =
 * the leading and trailing rows of each tile the forward solve's summaries
 * read (tdt_green_support rounded up to multiples of 64; for a general
 * plan whose size is a multiple of the tile, the widest supports of the
 * tiles' own inverses), rows4[2], rows4[3] the same for the adjoint (the
 * rows of T^T); 0, 0 when the pass reads whole tiles (the supports would
 * cover a quarter of the tile or more: weak dominance) or the plan has no
 * such pass (one tile, varlen or strided plans, or a general plan with a
 * ragged last tile).  Errors: null arguments -> TDT_ERR_INVALID_ARG. */
tdt_status_t tdt_plan_green_support(tdt_plan_t plan, int64_t *rows4);

/* Host-only: the interface merge of two adjacent segments, in double, as the
 * kernels compute it.  seg = (y_first, y_last, phi_first, phi_last,
 * chi_first, chi_last) of the left (l) and right (r) segment; out = the
 * merged six values.  Returns TDT_ERR_SINGULAR if the merge divides by 0. */
tdt_status_t tdt_segment_merge(const double *l, const double *r, double *out);

/* Measurement support.  While enabled (enable != 0), every solve of the plan
 * that is not being captured records HIP events on its stream around its
 * three kernel groups: the first pass over tiles (tile summaries), the
 * interface pass across tiles, and the final pass (solve and store).  Where
 * every multi-tile system has at most 64 tiles the final pass runs the
 * interface pass itself, and the interface group is empty (two events with
 * nothing between them); a small series of whole tiles (at most 256 in all)
 * is solved by the final pass alone, and the first-pass group is empty too.
 * tdt_plan_profile_read synchronises the device, returns in ms3[0..2] the
 * summed milliseconds of the three groups over the recorded solves and in
 * *nsolves their number, and clears the record.  Disabling clears it too. */
tdt_status_t tdt_plan_profile(tdt_plan_t plan, int enable);
tdt_status_t tdt_plan_profile_read(tdt_plan_t plan, double *ms3, int64_t *nsolves);

/* Launch-shape options of a plan.  None of them changes what is computed;
 * they trade how the work is spread over the device.
 *   TDT_OPT_WHOLE_MAX_TILES  varlen plans: systems of at most this many tiles
 *       (8192 rows each) are solved whole by one workgroup each, so that a
 *       batch of such systems takes a single launch whose second read of
 *       every tile comes from cache; larger systems go through the
 *       tile-parallel path (first pass, interface pass, final pass; the
 *       final pass runs the interface pass itself when every such system
 *       has at most 64 tiles).  0..16, default 8; 0 sends every multi-tile
 *       system through the tile-parallel path.
 *   TDT_OPT_WG_PER_CU        0 (default): the tile kernels launch one
 *       workgroup per tile and the other kernels as many workgroups as fit
 *       at once; k > 0: every kernel runs at most k persistent workgroups
 *       per compute unit, each looping over its share of the work.
 *   TDT_OPT_MAX_REFINE       TDT_F32_REFINE: most float solves per tile
 *       (1..100, default 40).
 *   TDT_OPT_SHAPE            work shape of the tile kernels: 0 = blocks of
 *       16 rows per lane and 512 lanes per workgroup (tiles of 8192 rows,
 *       default), 1 = 8 rows x 512 lanes (tiles of 4096), 2 = 16 rows x 256
 *       lanes (tiles of 4096).  Setting it rebuilds the plan's tables for the
 *       new block length (blocking; results change only by rounding). */
typedef enum {
    TDT_OPT_WHOLE_MAX_TILES = 0,
    TDT_OPT_WG_PER_CU = 1,
    TDT_OPT_MAX_REFINE = 2,
    TDT_OPT_SHAPE = 3
} tdt_option_t;

/* Set / read an option.  Errors: unknown option, value out of range, or
 * TDT_OPT_WHOLE_MAX_TILES on a series plan -> TDT_ERR_INVALID_ARG.  Setting
 * TDT_OPT_WHOLE_MAX_TILES, TDT_OPT_WG_PER_CU (varlen) or TDT_OPT_SHAPE
 * rebuilds the plan's work lists or tables (blocking; a reservation made
 * with tdt_plan_reserve is renewed) and must not happen while a solve of the
 * plan may run or is being captured. */
tdt_status_t tdt_plan_set_option(tdt_plan_t plan, tdt_option_t opt, int64_t value);
tdt_status_t tdt_plan_get_option(tdt_plan_t plan, tdt_option_t opt, int64_t *value);

/* Autotuner: times the candidate work and launch shapes (TDT_OPT_SHAPE,
 * TDT_OPT_WG_PER_CU, and TDT_OPT_WHOLE_MAX_TILES for varlen plans) on the
 * caller's data with HIP events on `stream`, and keeps the fastest.  F, X (and M for a series
 * plan; ignored for varlen) as for tdt_solve / tdt_solve_varlen; X is
 * overwritten by the trial solves (it ends holding the solution).
 * Synchronises the stream; refused while it is being captured
 * (TDT_ERR_CAPTURE).  The choice is cached in a JSON file keyed by device
 * (architecture, compute units), plan kind, dtype and problem size (sizes
 * rounded up to powers of two): the file named by the environment variable
 * TDT_TUNE_CACHE, else $HOME/.cache/tdt/autotune.json.  A cached choice is
 * applied without timing.  flags: TDT_TUNE_NO_CACHE neither reads nor
 * writes the file; TDT_TUNE_FORCE times again and replaces the entry;
 * TDT_TUNE_ADJOINT times each trial as a solve followed by
 * tdt_solve_backward (gX = F, into buffers the tuner allocates and frees),
 * for plans used in training loops (its own cache entry).
 * *best_ms (may be NULL): the chosen shape's time per solve (0 when taken
 * from the cache). */
#define TDT_TUNE_NO_CACHE 1
#define TDT_TUNE_FORCE 2
#define TDT_TUNE_ADJOINT 4
tdt_status_t tdt_plan_autotune(tdt_plan_t plan, const void *F, void *X, int64_t M,
                               hipStream_t stream, int flags, double *best_ms);

/* Compile-time layout facts of this build: block length B and threads per
 * workgroup for double and float data, and the tile length. */
tdt_status_t tdt_build_info(int *block_f64, int *block_f32, int *wg_threads,
                            int64_t *tile_len);

#ifdef __cplusplus
}
#endif
#endif /* TDT_H */
