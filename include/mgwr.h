/*
 * mgwr.h -- C ABI of the MI355X (gfx950) multigrid waveform relaxation
 * (MGWR) solver for the time-fractional heat equation
 *     D_t^alpha u - Laplace(u) = f  on (0, L)^dims x (0, T],
 *     u = 0 on the boundary, u(., 0) = g,
 * discretised with the L1 scheme in time and central differences in space
 * (Gaspar & Rodrigo, arXiv:1608.05400, Section 2 and Section 6), and solved
 * by Algorithm 1 (Section 3): red-black waveform relaxation that solves one
 * lower-triangular Toeplitz system along all M time levels per spatial point,
 * coarsening in space only, full weighting and linear/bilinear interpolation.
 *
 * Array conventions (every array argument is a DEVICE pointer, FP64,
 * contiguous, owned by the caller; the library never keeps a pointer after
 * the call returns):
 *   dims = 1: f, u, r are [M][N]; element (m, n-1) is the value at node
 *             x_n = n h (n = 1..N, h = L/(N+1)) and time t_{m+1} = (m+1) T/M;
 *             g (the initial condition, "u0") is [N].
 *   dims = 2: f, u, r are [M][N][N]; element (m, l-1, n-1) is the value at
 *             (x_n, y_l, t_{m+1}), x fastest; g is [N][N].
 *   t_0 is not stored: it is given by g.  g == NULL means g = 0.
 *
 * Work is issued on the handle's stream (mgwr_set_stream; default: the null
 * stream) and is stream-ordered with the caller's work on that stream.
 * mgwr_solve synchronises the stream before it returns (it reads residual
 * norms); the other calls are asynchronous unless stated.
 *
 * Return codes: MGWR_OK (0) on success; a positive code is a completed call
 * with a warning (u holds the last iterate); a negative code is an error, in
 * which case nothing was written to the output arrays unless stated and
 * mgwr_last_error() describes it.  A handle is not thread-safe; distinct
 * handles are independent.
 */
#ifndef MGWR_H
#define MGWR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgwr_ctx *mgwr_t;
typedef struct mgwr_batch_ctx *mgwr_batch_t;

enum mgwr_status {
    MGWR_OK = 0,
    MGWR_NOT_CONVERGED = 1, /* maxit cycles done before the tolerance was met          */
    MGWR_STAGNATED = 2,     /* residual stopped decreasing above the tolerance         */
    MGWR_EINVAL = -1,       /* invalid argument (sizes, alpha, T, dims, NULL pointers)  */
    MGWR_ENOMEM = -2,       /* device allocation failed                                 */
    MGWR_EDEVICE = -3,      /* HIP runtime error                                        */
    MGWR_ENONFINITE = -4,   /* NaN or Inf in the residual (input or divergence)         */
    MGWR_EDIVERGED = -5     /* residual grew beyond 1e6 times its initial value         */
};

/* Arithmetic of the V-cycle. */
enum mgwr_precision {
    MGWR_FP64 = 0,          /* Algorithm 1 applied to u in FP64 ("plain")                 */
    MGWR_MIXED_FP32 = 1,    /* refinement: FP64 residual, V-cycle on the error in FP32    */
    MGWR_MIXED_BF16X3 = 2,  /* refinement: FP64 residual, V-cycle on the error in FP32
                               storage with Toeplitz products as three BF16 MFMA passes
                               (hi*hi + hi*lo + lo*hi) accumulated in FP32               */
    MGWR_FP64_REFINED = 3   /* refinement with an FP64 V-cycle on the error            */
};

enum mgwr_norm { MGWR_NORM_MAX = 0, MGWR_NORM_L2 = 1 };

/* Smoother line solve (Section 5.2): all solve (T_M + sigma I) x = b along
 * every time line of one colour exactly (up to rounding). */
enum mgwr_smoother {
    MGWR_SMOOTH_INVERSE = 0, /* one causal Toeplitz product with the precomputed first
                                column of (T_M + sigma I)^{-1}                        */
    MGWR_SMOOTH_DC = 1,      /* divide-and-conquer blocked forward substitution: rows cut
                                into base blocks of dc_block rows, each solved with the
                                inverse of the leading block; after base block j the rows
                                of the D&C node split at j + 1 get the history of the
                                node's top half as one full Toeplitz-block product     */
    MGWR_SMOOTH_AUTO = 2     /* per level, whichever of the two the autotuner timed
                                fastest (MGWR_SMOOTH_INVERSE until mgwr_autotune)      */
};

typedef struct {
    int nu1, nu2;       /* pre-/post-smoothing steps of Algorithm 1 (default 1, 1)          */
    int gamma;          /* coarse cycles per level: 1 = V, 2 = W (default 1)                 */
    int maxit;          /* maximum cycles in mgwr_solve (default 100)                        */
    int norm;           /* enum mgwr_norm (default MGWR_NORM_MAX)                            */
    int warm_start;     /* mgwr_solve: 1 = u already holds the initial iterate (default 0:
                           u^0 = g at every time level, Section 3)                         */
    int precision;      /* enum mgwr_precision (default MGWR_FP64)                           */
    int first_colour;   /* colour relaxed first: 0 = even n (2D: n + l even), as ordered in
                           the text of Section 3; 1 = odd n first (default 0)              */
    int smoother;       /* enum mgwr_smoother (default MGWR_SMOOTH_INVERSE)                  */
    int dc_block;       /* base block of MGWR_SMOOTH_DC: a multiple of 128, or 0 = the
                           autotuner's per-level choice (1024 before mgwr_autotune); a block
                           of M rows or more is the inverse-column solve                  */
    double L;           /* domain length (default 1)                                         */
    double stall;       /* mgwr_solve stops with MGWR_STAGNATED when a cycle reduces the
                           residual by less than this factor (default 0.5; 0 disables)      */
    int graph;          /* 1 = record each outer iteration of mgwr_solve /
                           mgwr_batch_solve once per set of arguments and replay it as a
                           HIP graph; 0 = issue every launch each time (default 1)          */
    int fft;            /* FP64 Toeplitz products (the FP64 residual, FP64 smoother and
                           FP64 cycles) as circulant products by FFT (Section 5.1) instead of
                           dense matrix-core products: 0 = never, 1 = per level as the
                           autotuner chose (before tuning: when M >= 1024), 2 = always
                           (M >= 32).  The two routes agree to rounding (default 1)       */
    int inner_cycles;   /* refinement precisions: cycles of the error equation per
                           refinement step, 1..8 (default 1).  More cycles per step save
                           FP64 residuals but the later cycles of a step work from a
                           residual with the FFT route's FP32 rounding, which is relative
                           to the largest values of a time line: on the 1D N = 4095,
                           M = 16384 problems two per step took 14 cycles against 10   */
} mgwr_options;

typedef struct {
    int iters;          /* cycles done (refinement precisions: refinement steps, each of
                           inner_cycles cycles)                                            */
    int status;         /* the return code of mgwr_solve                                      */
    double r0;          /* norm of the initial residual                                       */
    double rk;          /* norm of the final residual                                         */
    double relres;      /* rk / r0                                                            */
    double mean_factor; /* (rk / r0)^(1/iters)  (Section 7, mean convergence factor)          */
    double hist[128];   /* residual norms after 0..min(iters,127) cycles                      */
} mgwr_info;

/* Nonlinear problem of Section 7 (anomalous diffusion in porous media):
 *   D_t^alpha u = (D(u) u_x)_x + c u_x + f on (0, 1) x (0, T],
 * zero initial and Dirichlet values, D(u) = 1 + q u^2 (the paper: q = 1,
 * c = 1, f = 1).  Discretised by the L1 scheme in time, the diffusion term
 * with half-point coefficients (D(u_{n+-1}) + D(u_n)) / 2 and the convection
 * term upwinded (forward difference: c >= 0).  Solved by the waveform
 * relaxation FAS method (Section 7): V(nu1, nu2) cycles, red-black nonlinear
 * Gauss-Seidel smoothing (each point's time line solved with its neighbours
 * fixed, level by level by Newton's method), full weighting of residual and
 * solution, linear interpolation of the correction; colour 0 = even n,
 * first_colour relaxed first (1 reproduces Table 5), starting from u = 0,
 * until the max-norm residual is reduced by tol or maxit cycles are done.
 * N = 2^k - 1, 1 <= M <= 4096; f, u: DEVICE [M][N] FP64 (u is overwritten with the iterate;
 * the caller owns both); stream: a hipStream_t or NULL.  The call allocates
 * its hierarchy on the device, frees it before returning and synchronises
 * the stream.  Returns MGWR_OK, MGWR_NOT_CONVERGED, or a negative code
 * (MGWR_EINVAL for bad arguments, MGWR_ENONFINITE for a NaN/Inf residual);
 * info (host, may be NULL) receives iterations and residual history. */
int mgwr_fas_solve(int N, int M, double alpha, double T, double c, double q, int nu1, int nu2,
                   int first_colour, const double *f, double *u, double tol, int maxit, void *stream,
                   mgwr_info *info);

/* count problems of the nonlinear problem above with the same N, M, T, c, q
 * and cycle, each with its own alpha[i], f[i] and u[i] (host arrays of count
 * values / device pointers): each runs on a stream of its own, created by the
 * call and ordered after the work already on stream, so that the problems'
 * kernels overlap; every problem stops by its own test.  infos (host, may be
 * NULL) receives count records.  Returns MGWR_ENONFINITE if any problem's
 * residual is not finite, else MGWR_NOT_CONVERGED if any did not converge,
 * else MGWR_OK; MGWR_EINVAL for bad arguments (nothing written). */
int mgwr_fas_solve_batch(int count, int N, int M, const double *alpha, double T, double c, double q,
                         int nu1, int nu2, int first_colour, const double *const *f, double *const *u,
                         double tol, int maxit, void *stream, mgwr_info *infos);

/* Fill *o with the defaults listed above.  Host only; never fails. */
int mgwr_default_options(mgwr_options *o);

/* L1 weights of the time discretisation (Section 2, L1 scheme; Section 5,
 * first column of T_M): *c = tau^-alpha / Gamma(2 - alpha) and
 * r[i-1] = c (d_i - d_{i-1}), i = 1..M, d_k = k^(1-alpha) - (k-1)^(1-alpha),
 * d_0 = 0, d_1 = 1.  Host only (no device use).  r: host array of M doubles.
 * Returns MGWR_EINVAL on bad sizes or alpha outside (0, 1]. */
int mgwr_l1_weights(int M, double alpha, double T, double *c, double *r);

/* Create a solver for N interior points per dimension (N = 2^k - 1, k >= 1,
 * so that coarsening reaches one point, Section 1 and Section 3), M >= 1 time
 * steps, order 0 < alpha <= 1, final time T > 0, dims in {1, 2}.  Computes
 * the L1 weights and, for every level, the first column of the inverse of
 * T_M + sigma_l I (Section 5.2), and allocates the device hierarchy on the
 * current HIP device.  opts may be NULL (defaults).  Synchronous. */
int mgwr_create(int N, int M, double alpha, double T, int dims, mgwr_t *out);
int mgwr_create_ex(int N, int M, double alpha, double T, int dims, const mgwr_options *opts,
                   mgwr_t *out);
int mgwr_destroy(mgwr_t h);

/* Change options (allocates the buffers the new precision needs). */
int mgwr_set_options(mgwr_t h, const mgwr_options *opts);
int mgwr_get_options(mgwr_t h, mgwr_options *opts);

/* hip_stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
int mgwr_set_stream(mgwr_t h, void *hip_stream);

/* `sweeps` red-black waveform-relaxation steps (Section 3, eq. red-black;
 * Section 6, eq. red-black_2d) on the finest level, in place on u: for each
 * colour in turn, every point p of that colour gets the solution x of
 * (T_M + sigma I) x = f_p + c d g_p + (sum of neighbours of p)/h^2.
 * Arithmetic of options.precision, as in the cycles of mgwr_solve:
 * MGWR_FP64 and MGWR_FP64_REFINED entirely in FP64; MGWR_MIXED_FP32 and
 * MGWR_MIXED_BF16X3 with the history part of each line solve (the product
 * with the inverse column without its first entry) in FP32 or split BF16
 * (levels with fewer than 128 points of a colour in FP32; on the FFT route
 * FP32 arithmetic, or FP64 where c > 0.1 sigma), its diagonal term
 * lambda_0 b and every grid function in FP64.  This is the smoothing step of
 * the inner cycles of the refinement, exposed so that it can be checked on
 * its own: in those precisions f and u are copied into the refinement's
 * internal hierarchy (its levels stored split by colour) and u back. */
int mgwr_smooth(mgwr_t h, const double *f, const double *g, double *u, int sweeps);

/* Residual r = f + c d_m g - T_M u - A_h u of the discrete problem (Section 2,
 * eq. discrete_model_IVP_1; Section 6), in FP64.  If norms != NULL (host,
 * 2 doubles) it receives {max |r|, ||r||_2} and the call synchronises. */
int mgwr_residual(mgwr_t h, const double *f, const double *g, const double *u, double *r,
                  double *norms);

/* One cycle of Algorithm 1 (V or W per options.gamma) on u in place, in the
 * arithmetic of options.precision (as mgwr_smooth; the residuals of the
 * levels below the finest as well).  In the refinement precisions the
 * residual before restriction is computed at the first colour's points only
 * on the FFT route (after a red-black sweep the other colour's residual is
 * zero up to the rounding of its line solves), as in the inner cycles of
 * mgwr_solve; MGWR_FP64 computes it everywhere. */
int mgwr_vcycle(mgwr_t h, const double *f, const double *g, double *u);

/* Iterate until ||r_k|| <= tol ||r_0|| (norm per options; Section 7 uses a
 * reduction by 1e-10), maxit, or stagnation.  u receives the last iterate.
 * info may be NULL.  Synchronises the stream. */
int mgwr_solve(mgwr_t h, const double *f, const double *g, double *u, double tol,
               mgwr_info *info);

/* C = X B, B and C device [M][ldb]/[M][ldc] FP64 with P columns, where X is
 * the lower-triangular Toeplitz matrix T_M (which = -1) or the inverse of
 * T_M + sigma_l I on level `which` >= 0 (0 = coarsest), applied in the
 * arithmetic `precision` (enum mgwr_precision; FP64_REFINED is FP64).
 * Exposes the Toeplitz product kernels for testing. */
int mgwr_toeplitz_apply(mgwr_t h, int which, int precision, const double *B, int ldb, int P,
                        double *C, int ldc);

/* Bytes of the device scratch of mgwr_toeplitz_apply_static (one static
 * array per GPU, held from library load until the process ends). */
#define MGWR_STATIC_SCRATCH_BYTES (64u << 20)

/* mgwr_toeplitz_apply without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same products on the same kernels,
 * with everything beyond B and C (the low-precision copy of the operand, the
 * split-K partial sums, the FFT route's work arrays) in a static device
 * array of MGWR_STATIC_SCRATCH_BYTES per GPU instead of the handle's
 * buffers or temporaries.  It calls no hipMalloc, hipFree or stream
 * synchronisation; the work is queued on the handle's stream.  Rejected with
 * MGWR_EINVAL (nothing launched): FP32 operands of more than
 * MGWR_STATIC_SCRATCH_BYTES (4 M P bytes), split-BF16 operands of more than
 * that (4 Mpad ldp bytes, Mpad = M rounded up to 128, ldp = P rounded up to
 * 128), and FFT-route products whose one column pair does not fit half of
 * it (16 L bytes in FP64, 8 L in FP32, L the transform length >= 2M); larger
 * FFT-route products run in chunks of columns.  Every call on one GPU uses
 * that GPU's one array and leaves its contents behind (nothing in it needs
 * to start at zero): calls that overlap in time on one GPU, on any streams or
 * handles, race and give wrong results; order them on one stream. */
int mgwr_toeplitz_apply_static(mgwr_t h, int which, int precision, const double *B, int ldb, int P,
                               double *C, int ldc);

/* Host copy of the first column (M doubles) of T_M (which = -1) or of the
 * inverse of T_M + sigma_l I on level `which`. */
int mgwr_get_column(mgwr_t h, int which, double *out);

/* Number of levels (finest = levels - 1). */
int mgwr_levels(mgwr_t h);

/* ---- autotuner ----
 * Times one cycle of the error equation of the handle (its own buffers only:
 * no caller array is read or written) under candidate tile shapes of the
 * Toeplitz-product kernels, the FFT or dense route of the FP64 products per
 * level (options.fft = 1), and, when options.smoother is MGWR_SMOOTH_DC with
 * dc_block = 0 or MGWR_SMOOTH_AUTO, candidate D&C base blocks per level, and
 * keeps the fastest.  Handles of the same shape and options created later in
 * the process reuse the result; if the environment variable MGWR_TUNE_CACHE
 * names a file, results are also appended to it and read from it by later
 * processes (single handles; a malformed or unreadable file is ignored).
 * Synchronous; the choice is reported by mgwr_get_tuning. */
typedef struct {
    int tuned;            /* 1 once mgwr_autotune has run                                */
    int variant[2];       /* FP64 / FP32 product tile: -1 by size, 0 = 128x64, 1 = 256x64 */
    int split_target[3];  /* FP64 / FP32 / split-BF16 work items a lone launch aims for
                             (0 = default); fewer tiles than that split the K range     */
    int levels;
    int dc_block[32];     /* per level (0 = coarsest): 0 = inverse-column solve, else the
                             D&C base block in rows                                       */
    int fft[32];          /* per level: 1 = FP64 products by FFT, 0 = dense               */
    double ms_default;    /* cycle time with the default choices (ms)                    */
    double ms_tuned;      /* cycle time with the chosen ones (ms)                        */
} mgwr_tuning;
int mgwr_autotune(mgwr_t h);
int mgwr_get_tuning(mgwr_t h, mgwr_tuning *t);
/* Apply a tuning obtained from mgwr_get_tuning on a handle of the same shape
 * and options (for instance saved by an earlier process), instead of running
 * the autotuner.  MGWR_EINVAL if the level count differs or a field is out of
 * range (variant -1..1, split_target >= 0, dc_block 0 or a multiple of 128,
 * fft 0 or 1); the handle is then unchanged. */
int mgwr_set_tuning(mgwr_t h, const mgwr_tuning *t);

/* ---- batches of independent 1D or 2D problems (uneven N, M, alpha) ----
 * count problems; N[i], M[i], alpha[i], T[i] as for mgwr_create; all share
 * dims and opts.  f, g, u are host arrays of count device pointers (g may
 * be NULL or contain NULLs).  infos: host array of count mgwr_info (may be
 * NULL).  The problems are solved together: every stage of a cycle (colour
 * right-hand sides, Toeplitz products, residuals, transfers, norms) is ONE
 * launch over all problems still iterating, their product tiles ordered by
 * K extent; each problem stops by its own test, with the results mgwr_solve
 * would give it.  Returns the worst status over the problems (a negative
 * one if any failed; mgwr_last_error names the problem). */
int mgwr_batch_create(int count, const int *N, const int *M, const double *alpha,
                      const double *T, int dims, const mgwr_options *opts, mgwr_batch_t *out);
int mgwr_batch_solve(mgwr_batch_t b, const double *const *f, const double *const *g,
                     double *const *u, double tol, mgwr_info *infos);
int mgwr_batch_set_stream(mgwr_batch_t b, void *hip_stream);
/* The autotuner over the whole batch (one set of tile shapes and per-depth
 * D&C blocks for all problems, timed on a cycle of all of them). */
int mgwr_batch_autotune(mgwr_batch_t b);
int mgwr_batch_get_tuning(mgwr_batch_t b, int i, mgwr_tuning *t);
int mgwr_batch_destroy(mgwr_batch_t b);

/* ---- per-launch timing of the Toeplitz products (history GEMMs) ----
 * With profiling on, every Toeplitz-product launch of the handle (or batch)
 * is bracketed by HIP events recorded on its stream, and mgwr_solve issues
 * its launches one by one instead of replaying graphs.  kernel identifies
 * the kernel instantiation: (kind << 8) | (mode << 4) | epilogue, with kind
 * 0 = narrow (64x16 tiles), 1 = wide 128x64, 2 = wide 256x64, 3 = split-BF16
 * 256x128, 4 = FFT route (all passes of one product), 5 = FFT route with
 * the whole product in one kernel (FP64, M <= 2048); mode 0 = FP64, 1 = FP32,
 * 2 = split-BF16; epilogue 0 = store (residual product, D&C base block in
 * FP64, FP64 smoother on a level stored split by colour), 1 = colour scatter
 * (FP64 smoother, whole line solve, level in natural order), 3 = subtract
 * (D&C history update), 4 = add (D&C base block, or the history part of a
 * split level's smoother), 6 = residual (FFT route: the stencil part minus
 * the product, written as the residual), 7 = the same for a double-double
 * iterate, 8 = the residual at one colour's points (inner cycles of the
 * refinement after pre-smoothing), 9 = the same in 1D with colour 0 first,
 * written restricted to the coarse grid, 10 = the diagonal term plus the
 * history part into a split level's colour points (smoother, FP32 FFT
 * route).
 * A record covers one launch, possibly over several products (of several
 * problems): M and K are the largest of them, P the sum of their columns,
 * and flops, bytes and pass_bytes sums of per-product values.  ms covers
 * the product and, when its K range is split over several blocks, the
 * reduce kernel that applies its epilogue. */
typedef struct {
    int kernel, level, M, P, K;
    double flops;      /* algorithmic flops: multiply-adds of the products that are
                          not structurally zero, times 2                            */
    double ms;         /* elapsed time between the two events                      */
    double bytes;      /* the products' own HBM bytes: the operand read once (in the
                          precision it is handed over: 8 bytes FP64, 4 FP32 or split
                          BF16 hi + lo) plus, per output element, what the epilogue
                          must read and write: 8 (store), 16 (read-modify-write, or
                          the right-hand side read for the diagonal term and the
                          value written), 16 / 24 (residual: F and the result, and
                          the double-double low part / the other colour's neighbours) */
    double pass_bytes; /* FFT route: the bytes its passes move through the complex
                          work arrays on top of `bytes` (0 for the dense kernels)    */
    int products;      /* Toeplitz products in the launch                          */
} mgwr_kernel_record;

/* on != 0 clears the records and starts recording; on == 0 stops. */
int mgwr_profile_enable(mgwr_t h, int on);
/* Number of records (synchronises the handle's stream). */
int mgwr_profile_count(mgwr_t h);
int mgwr_profile_get(mgwr_t h, int i, mgwr_kernel_record *rec);
/* Name of the kernel function of a kernel id (as profilers print it). */
const char *mgwr_kernel_name(int kernel);
int mgwr_batch_profile_enable(mgwr_batch_t b, int on);
int mgwr_batch_profile_count(mgwr_batch_t b);
int mgwr_batch_profile_get(mgwr_batch_t b, int i, mgwr_kernel_record *rec);

/* Message of the last error on the calling thread ("" if none). */
const char *mgwr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGWR_H */
