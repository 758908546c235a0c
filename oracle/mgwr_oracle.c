/*
 * mgwr_oracle.c -- plain, slow CPU oracle in FP64 for multigrid waveform
 * relaxation (MGWR) applied to the time-fractional heat equation
 * (Gaspar & Rodrigo, "Multigrid waveform relaxation for the time-fractional
 * heat equation", arXiv:1608.05400).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or constant with the GPU
 * library.
 *
 * Conventions (all arrays are caller-owned, row-major, FP64):
 *   dims = 1: grid functions are [M][N]; entry (m, n-1) holds u_{n,m+1},
 *             n = 1..N (interior nodes x_n = n h, h = L/(N+1)), m = 0..M-1
 *             holds time level t_{m+1} = (m+1) tau, tau = T/M.
 *   dims = 2: grid functions are [M][N][N]; entry (m, l-1, n-1) holds
 *             u_{n,l,m+1}, x fastest.
 *   g is the initial condition at the interior nodes ([N] or [N][N]); NULL
 *   means g = 0.  Boundary values are zero (Section 2, Dirichlet data;
 *   Section 6 for 2D).
 *
 * Every function cites the passage of the paper it writes out.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* L1 weights.  Section 2, eqs. (L1_scheme1)-(L1_scheme2): the Caputo
 * derivative at t_m is approximated by
 *   c [ d_1 u_m - d_m u_0 + sum_{k=1}^{m-1} (d_{k+1} - d_k) u_{m-k} ],
 * c = tau^{-alpha} / Gamma(2 - alpha), d_k = k^{1-alpha} - (k-1)^{1-alpha}.
 * Section 5 writes the same operator as the lower-triangular Toeplitz matrix
 * T_M with first column r_i = c (d_i - d_{i-1}), d_0 = 0.
 *
 * Reading: d_k is evaluated as -k^b expm1(b log1p(-1/k)) (b = 1 - alpha) in
 * long double, which is the same number written so that the subtraction of
 * two nearly equal powers does not lose digits; d_1 = 1 for every alpha in
 * (0, 1] (so alpha = 1 is backward Euler).                                  */
static long double l1_d(long k, long double b)
{
    if (k <= 0) return 0.0L;
    if (k == 1) return 1.0L;
    return -powl((long double)k, b) * expm1l(b * log1pl(-1.0L / (long double)k));
}

/* c_out <- c;  d[0..M] <- d_0..d_M;  r[0..M-1] <- r_1..r_M. */
void orc_l1_coeffs(int M, double alpha, double T, double *c_out, double *d, double *r)
{
    long double b = 1.0L - (long double)alpha;
    long double tau = (long double)T / (long double)M;
    long double c = powl(tau, -(long double)alpha) / tgammal(2.0L - (long double)alpha);
    long double dprev = 0.0L;
    if (c_out) *c_out = (double)c;
    if (d) d[0] = 0.0;
    for (long k = 1; k <= M; ++k) {
        long double dk = l1_d(k, b);
        if (d) d[k] = (double)dk;
        if (r) r[k - 1] = (double)(c * (dk - dprev));
        dprev = dk;
    }
}

/* ------------------------------------------------------------------------ */
/* Small helpers shared by the oracle's own routines.                        */
typedef struct {
    int dims, N, M, npts;
    double h, L, c;
    double *r;   /* r_1..r_M */
    double *d;   /* d_0..d_M */
} orc_grid;

static void grid_init(orc_grid *G, int dims, int N, int M, double alpha, double T, double L)
{
    G->dims = dims; G->N = N; G->M = M; G->L = L;
    G->npts = (dims == 1) ? N : N * N;
    G->h = L / (double)(N + 1);
    G->r = (double *)malloc(sizeof(double) * (size_t)M);
    G->d = (double *)malloc(sizeof(double) * (size_t)(M + 1));
    orc_l1_coeffs(M, alpha, T, &G->c, G->d, G->r);
}
static void grid_free(orc_grid *G) { free(G->r); free(G->d); }

/* Value of grid function v (one time level, npts entries) at interior index
 * (n, l) in paper numbering; zero on and outside the boundary. */
static double at1(const double *v, int N, int n)
{
    return (n >= 1 && n <= N) ? v[n - 1] : 0.0;
}
static double at2(const double *v, int N, int n, int l)
{
    return (n >= 1 && n <= N && l >= 1 && l <= N) ? v[(size_t)(l - 1) * N + (n - 1)] : 0.0;
}

/* (A_h v)(p) for the 3-point (Section 2, eq. discrete_model_IVP_1) or
 * 5-point (Section 6, Delta_h) negative Laplacian at flat point index p. */
static double apply_Ah(const orc_grid *G, const double *v, int p)
{
    double ih2 = 1.0 / (G->h * G->h);
    if (G->dims == 1) {
        int n = p + 1;
        return (2.0 * at1(v, G->N, n) - at1(v, G->N, n - 1) - at1(v, G->N, n + 1)) * ih2;
    } else {
        int n = p % G->N + 1, l = p / G->N + 1;
        return (4.0 * at2(v, G->N, n, l) - at2(v, G->N, n - 1, l) - at2(v, G->N, n + 1, l)
                - at2(v, G->N, n, l - 1) - at2(v, G->N, n, l + 1)) * ih2;
    }
}

/* Sum of the spatial neighbours of point p (the off-diagonal part N_h of the
 * splitting A_h = M_h - N_h, times h^2). */
static double nbr_sum(const orc_grid *G, const double *v, int p)
{
    if (G->dims == 1) {
        int n = p + 1;
        return at1(v, G->N, n - 1) + at1(v, G->N, n + 1);
    } else {
        int n = p % G->N + 1, l = p / G->N + 1;
        return at2(v, G->N, n - 1, l) + at2(v, G->N, n + 1, l)
             + at2(v, G->N, n, l - 1) + at2(v, G->N, n, l + 1);
    }
}

/* Colour of flat point p: 0 (red) if n (1D) or n + l (2D) is even, else 1.
 * Section 3, eq. (red-black): even points are visited first; Section 6,
 * eq. (red-black_2d): n + l even first. */
static int colour_of(const orc_grid *G, int p)
{
    if (G->dims == 1) return ((p + 1) % 2 == 0) ? 0 : 1;
    int n = p % G->N + 1, l = p / G->N + 1;
    return ((n + l) % 2 == 0) ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Residual of the discrete problem.  Section 2, eqs. (discrete_model_IVP_1-3)
 * and Section 6, eqs. (discrete_model_IVP_2d_1-3):
 *   R_{p,m} = f_{p,m} + c d_m g_p - (T_M u_p)_m - (A_h u_{.,m})_p
 * where the term c d_m g_p is the -c d_m u_{n,0} part of the L1 formula moved
 * to the right-hand side.  Written as the plain double loop.               */
void orc_residual(int dims, int N, int M, double alpha, double T, double L,
                  const double *f, const double *g, const double *u, double *R)
{
    orc_grid G; grid_init(&G, dims, N, M, alpha, T, L);
    int P = G.npts;
#pragma omp parallel for schedule(static)
    for (int m = 0; m < M; ++m) {
        const double *um = u + (size_t)m * P;
        for (int p = 0; p < P; ++p) {
            double hist = 0.0;
            for (int j = 0; j <= m; ++j) hist += G.r[m - j] * u[(size_t)j * P + p];
            double gp = g ? g[p] : 0.0;
            R[(size_t)m * P + p] = f[(size_t)m * P + p] + G.c * G.d[m + 1] * gp
                                   - hist - apply_Ah(&G, um, p);
        }
    }
    grid_free(&G);
}

/* One half-sweep of red-black waveform relaxation.  Section 3, eq. (red-black)
 * (1D) and Section 6, eq. (red-black_2d) (2D): for every point p of the given
 * colour, solve along the whole time line
 *   (T_M + sigma I) x = f_p + c d g_p + (sum of the neighbours of p)/h^2,
 * sigma = 2/h^2 (1D) or 4/h^2 (2D), with the current neighbour values, by
 * plain forward substitution, and store x as the new u_p.                   */
static void half_sweep_grid(const orc_grid *G, int colour, const double *f, const double *g, double *u)
{
    int P = G->npts, M = G->M;
    double ih2 = 1.0 / (G->h * G->h);
    double sigma = (G->dims == 1 ? 2.0 : 4.0) * ih2;
#pragma omp parallel
    {
        double *b = (double *)malloc(sizeof(double) * (size_t)M);
        double *x = (double *)malloc(sizeof(double) * (size_t)M);
#pragma omp for schedule(dynamic, 4)
        for (int p = 0; p < P; ++p) {
            if (colour_of(G, p) != colour) continue;
            double gp = g ? g[p] : 0.0;
            for (int m = 0; m < M; ++m)
                b[m] = f[(size_t)m * P + p] + G->c * G->d[m + 1] * gp
                       + nbr_sum(G, u + (size_t)m * P, p) * ih2;
            for (int m = 0; m < M; ++m) {
                double s = b[m];
                for (int j = 0; j < m; ++j) s -= G->r[m - j] * x[j];
                x[m] = s / (G->r[0] + sigma);
            }
            for (int m = 0; m < M; ++m) u[(size_t)m * P + p] = x[m];
        }
        free(b); free(x);
    }
}

void orc_half_sweep(int dims, int N, int M, double alpha, double T, double L, int colour,
                    const double *f, const double *g, double *u)
{
    orc_grid G; grid_init(&G, dims, N, M, alpha, T, L);
    half_sweep_grid(&G, colour, f, g, u);
    grid_free(&G);
}

/* Full-weighting restriction of a fine grid function (N_f points per
 * dimension) to the coarse grid (N_c = (N_f - 1)/2), at every time level.
 * Section 3 (standard full weighting) and Section 6 (its 2D form): coarse
 * node J sits on fine node 2J; 1D weights [1 2 1]/4, 2D the tensor product
 * [1 2 1]^T [1 2 1]/16.                                                    */
void orc_restrict(int dims, int Nf, int M, const double *rf, double *rc)
{
    int Nc = (Nf - 1) / 2;
    if (dims == 1) {
        for (int m = 0; m < M; ++m) {
            const double *v = rf + (size_t)m * Nf;
            for (int J = 1; J <= Nc; ++J)
                rc[(size_t)m * Nc + (J - 1)] =
                    0.25 * (at1(v, Nf, 2 * J - 1) + 2.0 * at1(v, Nf, 2 * J) + at1(v, Nf, 2 * J + 1));
        }
    } else {
        static const double w[3] = {1.0, 2.0, 1.0};
        for (int m = 0; m < M; ++m) {
            const double *v = rf + (size_t)m * Nf * Nf;
            for (int J = 1; J <= Nc; ++J)
                for (int I = 1; I <= Nc; ++I) {
                    double s = 0.0;
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a)
                            s += w[a + 1] * w[b + 1] * at2(v, Nf, 2 * I + a, 2 * J + b);
                    rc[(size_t)m * Nc * Nc + (size_t)(J - 1) * Nc + (I - 1)] = s / 16.0;
                }
        }
    }
}

/* Linear (1D) / bilinear (2D) interpolation of a coarse grid function to the
 * fine grid, added to uf.  Section 3 and Section 6: coarse node J coincides
 * with fine node 2J; an odd fine node takes the mean of its two coarse
 * neighbours (1D), or of its two or four coarse neighbours (2D); coarse
 * values on the boundary are zero.                                          */
void orc_prolong_add(int dims, int Nc, int M, const double *ec, double *uf)
{
    int Nf = 2 * Nc + 1;
    if (dims == 1) {
        for (int m = 0; m < M; ++m) {
            const double *v = ec + (size_t)m * Nc;
            for (int n = 1; n <= Nf; ++n) {
                double e = (n % 2 == 0) ? at1(v, Nc, n / 2)
                                        : 0.5 * (at1(v, Nc, (n - 1) / 2) + at1(v, Nc, (n + 1) / 2));
                uf[(size_t)m * Nf + (n - 1)] += e;
            }
        }
    } else {
        for (int m = 0; m < M; ++m) {
            const double *v = ec + (size_t)m * Nc * Nc;
            for (int l = 1; l <= Nf; ++l)
                for (int n = 1; n <= Nf; ++n) {
                    /* coarse x-neighbours of n and y-neighbours of l with weights */
                    int xa = n / 2, xb = (n + 1) / 2;      /* equal when n is even */
                    int ya = l / 2, yb = (l + 1) / 2;
                    double e = 0.25 * (at2(v, Nc, xa, ya) + at2(v, Nc, xb, ya)
                                       + at2(v, Nc, xa, yb) + at2(v, Nc, xb, yb));
                    uf[(size_t)m * Nf * Nf + (size_t)(l - 1) * Nf + (n - 1)] += e;
                }
        }
    }
}

/* One cycle of Algorithm 1 (WRMG, Section 3) on a level with N points per
 * dimension, pre-/post-smoothing nu1/nu2, gamma coarse cycles.  One
 * smoothing step is a half-sweep of colour `first` followed by one of the
 * other colour (first = 0: even n, resp. n + l even, as the text of Section 3
 * orders them).  The coarse operator is the same L1 time operator plus A_{2h}
 * rediscretised with twice the mesh size; the coarse problem has zero
 * initial error.  On the coarsest level (N = 1) one sweep over both colours
 * is the exact solve of the single time line.                               */
static void vcycle_rec(int dims, int N, int M, double alpha, double T, double L,
                       int nu1, int nu2, int gamma, int first,
                       const double *f, const double *g, double *u)
{
    orc_grid G; grid_init(&G, dims, N, M, alpha, T, L);
    size_t sz = (size_t)M * G.npts;
    int c0 = first ? 1 : 0, c1 = 1 - c0;
    if (N == 1) {
        half_sweep_grid(&G, c0, f, g, u);
        half_sweep_grid(&G, c1, f, g, u);
        grid_free(&G);
        return;
    }
    for (int i = 0; i < nu1; ++i) { half_sweep_grid(&G, c0, f, g, u); half_sweep_grid(&G, c1, f, g, u); }
    double *R = (double *)malloc(sizeof(double) * sz);
    orc_residual(dims, N, M, alpha, T, L, f, g, u, R);
    int Nc = (N - 1) / 2;
    size_t szc = (size_t)M * ((dims == 1) ? Nc : Nc * Nc);
    double *fc = (double *)malloc(sizeof(double) * szc);
    double *ec = (double *)calloc(szc, sizeof(double));
    orc_restrict(dims, N, M, R, fc);
    for (int k = 0; k < gamma; ++k)
        vcycle_rec(dims, Nc, M, alpha, T, L, nu1, nu2, gamma, first, fc, NULL, ec);
    orc_prolong_add(dims, Nc, M, ec, u);
    for (int i = 0; i < nu2; ++i) { half_sweep_grid(&G, c0, f, g, u); half_sweep_grid(&G, c1, f, g, u); }
    free(R); free(fc); free(ec);
    grid_free(&G);
}

void orc_vcycle(int dims, int N, int M, double alpha, double T, double L,
                int nu1, int nu2, int gamma, int first,
                const double *f, const double *g, double *u)
{
    vcycle_rec(dims, N, M, alpha, T, L, nu1, nu2, gamma, first, f, g, u);
}

/* Max norm and Euclidean norm of a residual. */
static void norms(const double *R, size_t n, double *nmax, double *n2)
{
    double a = 0.0, s = 0.0;
    for (size_t i = 0; i < n; ++i) { double v = fabs(R[i]); if (v > a) a = v; s += R[i] * R[i]; }
    *nmax = a; *n2 = sqrt(s);
}

/* MGWR iteration (Algorithm 1 repeated) from the initial iterate u^0 = g at
 * every time level (Section 3, after eq. GS_ODEs), stopped when the residual
 * has been reduced by the factor tol (Section 7: a reduction of the initial
 * residual by 1e-10).  norm = 0: max norm; 1: Euclidean.  Returns the number
 * of cycles done; hist[0..its] receives the residual norms.               */
int orc_mg_solve(int dims, int N, int M, double alpha, double T, double L,
                 int nu1, int nu2, int gamma, int first, int norm, double tol, int maxit, int warm,
                 const double *f, const double *g, double *u, double *hist)
{
    int P = (dims == 1) ? N : N * N;
    size_t sz = (size_t)M * P;
    if (!warm)
        for (int m = 0; m < M; ++m)
            for (int p = 0; p < P; ++p) u[(size_t)m * P + p] = g ? g[p] : 0.0;
    double *R = (double *)malloc(sizeof(double) * sz);
    double r0 = 0.0;
    int it = 0;
    for (;;) {
        double nmax, n2;
        orc_residual(dims, N, M, alpha, T, L, f, g, u, R);
        norms(R, sz, &nmax, &n2);
        double rn = norm ? n2 : nmax;
        if (hist) hist[it] = rn;
        if (it == 0) r0 = rn;
        if (rn <= tol * r0 || it >= maxit) break;
        orc_vcycle(dims, N, M, alpha, T, L, nu1, nu2, gamma, first, f, g, u);
        ++it;
    }
    free(R);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Exact solution of the discrete system by sequential time stepping: at each
 * level t_m the L1 history sum (all earlier levels, Section 2, eq.
 * L1_scheme2) goes to the right-hand side and the remaining spatial problem
 *   (r_1 I + A_h) u_{.,m} = f_{.,m} + c d_m g - sum_{j<m} r_{m-j+1} u_{.,j}
 * is solved directly: 1D by the Thomas algorithm (tridiagonal, diagonally
 * dominant, no pivoting); 2D by a discrete sine transform along y (the sine
 * vectors are eigenvectors of the 1D Dirichlet second difference) followed
 * by one tridiagonal solve along x per sine mode and the inverse transform.
 * Cost O(P M^2) for the history plus the spatial solves.  Only the first
 * Mstop levels are computed (Mstop <= 0 means all M).                       */
static void thomas(int n, double diag, double off, const double *rhs, double *x, double *cp)
{
    /* solves diag*x_i + off*(x_{i-1} + x_{i+1}) = rhs_i, x_0 = x_{n+1} = 0 */
    double b = diag;
    cp[0] = off / b;
    x[0] = rhs[0] / b;
    for (int i = 1; i < n; ++i) {
        double den = diag - off * cp[i - 1];
        cp[i] = off / den;
        x[i] = (rhs[i] - off * x[i - 1]) / den;
    }
    for (int i = n - 2; i >= 0; --i) x[i] -= cp[i] * x[i + 1];
}

void orc_direct_solve(int dims, int N, int M, double alpha, double T, double L,
                      const double *f, const double *g, double *u, int Mstop)
{
    orc_grid G; grid_init(&G, dims, N, M, alpha, T, L);
    int P = G.npts;
    double ih2 = 1.0 / (G.h * G.h);
    if (Mstop <= 0 || Mstop > M) Mstop = M;
    double *rhs = (double *)malloc(sizeof(double) * (size_t)P);
    double *S = NULL, *mu = NULL, *tmp = NULL;
    if (dims == 2) {
        S = (double *)malloc(sizeof(double) * (size_t)N * N);
        mu = (double *)malloc(sizeof(double) * (size_t)N);
        tmp = (double *)malloc(sizeof(double) * (size_t)N * N);
        for (int j = 1; j <= N; ++j) {
            double s = sin(j * M_PI / (2.0 * (N + 1)));
            mu[j - 1] = 4.0 * ih2 * s * s;
            for (int l = 1; l <= N; ++l) S[(size_t)(j - 1) * N + (l - 1)] = sin(j * l * M_PI / (N + 1));
        }
    }
    for (int m = 0; m < Mstop; ++m) {
        /* right-hand side with the history sum over all earlier levels */
#pragma omp parallel for schedule(static)
        for (int p = 0; p < P; ++p) {
            double s = f[(size_t)m * P + p] + G.c * G.d[m + 1] * (g ? g[p] : 0.0);
            for (int j = 0; j < m; ++j) s -= G.r[m - j] * u[(size_t)j * P + p];
            rhs[p] = s;
        }
        double *um = u + (size_t)m * P;
        if (dims == 1) {
            double *cp = (double *)malloc(sizeof(double) * (size_t)N);
            thomas(N, G.r[0] + 2.0 * ih2, -ih2, rhs, um, cp);
            free(cp);
        } else {
            /* forward sine transform along y: tmp[j][n] = sum_l S[j][l] rhs[l][n] */
#pragma omp parallel for schedule(static)
            for (int j = 0; j < N; ++j)
                for (int n = 0; n < N; ++n) {
                    double s = 0.0;
                    for (int l = 0; l < N; ++l) s += S[(size_t)j * N + l] * rhs[(size_t)l * N + n];
                    tmp[(size_t)j * N + n] = s;
                }
            /* one tridiagonal solve along x per sine mode j */
#pragma omp parallel
            {
                double *cp = (double *)malloc(sizeof(double) * (size_t)N);
                double *x = (double *)malloc(sizeof(double) * (size_t)N);
#pragma omp for schedule(static)
                for (int j = 0; j < N; ++j) {
                    thomas(N, G.r[0] + mu[j] + 2.0 * ih2, -ih2, tmp + (size_t)j * N, x, cp);
                    memcpy(tmp + (size_t)j * N, x, sizeof(double) * (size_t)N);
                }
                free(cp); free(x);
            }
            /* inverse transform: u[l][n] = 2/(N+1) sum_j S[l][j] tmp[j][n] */
#pragma omp parallel for schedule(static)
            for (int l = 0; l < N; ++l)
                for (int n = 0; n < N; ++n) {
                    double s = 0.0;
                    for (int j = 0; j < N; ++j) s += S[(size_t)l * N + j] * tmp[(size_t)j * N + n];
                    um[(size_t)l * N + n] = s * 2.0 / (N + 1);
                }
        }
    }
    free(rhs); free(S); free(mu); free(tmp);
    grid_free(&G);
}

/* ------------------------------------------------------------------------ */
/* Exact discrete solution for forcing that is a finite sum of sine modes.
 * The vectors sin(k pi x_n / L) are eigenvectors of A_h with eigenvalue
 * (4/h^2) sin^2(k pi h / (2L)) (the Fourier symbol of Section 4.1 taken at
 * the Dirichlet modes); in 2D the mode (k, j) has the sum of the two 1D
 * eigenvalues.  If f = sum_q s_q(t_m) phi_q and g = sum_q gq phi_q, then
 * u = sum_q v_q(t_m) phi_q with (T_M + lambda_q I) v_q = s_q + c d gq,
 * solved by forward substitution.  v is [K][M].                            */
void orc_modal_solve(int dims, int N, int M, double alpha, double T, double L,
                     int K, const int *kx, const int *ky, const double *s,
                     const double *gq, double *v)
{
    orc_grid G; grid_init(&G, dims, N, M, alpha, T, L);
    double h = G.h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < K; ++q) {
        double sx = sin(kx[q] * M_PI * h / (2.0 * L));
        double lam = 4.0 / (h * h) * sx * sx;
        if (dims == 2) {
            double sy = sin(ky[q] * M_PI * h / (2.0 * L));
            lam += 4.0 / (h * h) * sy * sy;
        }
        double gv = gq ? gq[q] : 0.0;
        double *x = v + (size_t)q * M;
        for (int m = 0; m < M; ++m) {
            double acc = s[(size_t)q * M + m] + G.c * G.d[m + 1] * gv;
            for (int j = 0; j < m; ++j) acc -= G.r[m - j] * x[j];
            x[m] = acc / (G.r[0] + lam);
        }
    }
    grid_free(&G);
}

/* Evaluate u = sum_q v_q(t_m) sin(kx pi x_n / L) [sin(ky pi y_l / L)] at
 * npt sample points given as (m, n[, l]) triples in paper numbering
 * (m = 1..M, n, l = 1..N).  pts is [npt][3] (l ignored in 1D).             */
void orc_modal_eval(int dims, int N, int M, double L, int K, const int *kx, const int *ky,
                    const double *v, int npt, const int *pts, double *out)
{
    double h = L / (double)(N + 1);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < npt; ++i) {
        int m = pts[3 * i], n = pts[3 * i + 1], l = pts[3 * i + 2];
        double s = 0.0;
        for (int q = 0; q < K; ++q) {
            double ph = sin(kx[q] * M_PI * n * h / L);
            if (dims == 2) ph *= sin(ky[q] * M_PI * l * h / L);
            s += v[(size_t)q * M + (m - 1)] * ph;
        }
        out[i] = s;
    }
}

/* Mittag-Leffler function E_a(z) = sum_k z^k / Gamma(a k + 1), the series by
 * which Section 7 defines it (exact solution E_a(-t^a) sin x of the first
 * test problem), summed term by term for each z[i] with |z[i]| <= 1: the
 * terms are then at most 1 in size and the sum ends when they fall below
 * e^-40 of that. */
void orc_mittag_leffler(double a, int n, const double *z, double *out)
{
    for (int i = 0; i < n; ++i) {
        if (z[i] == 0.0) {
            out[i] = 1.0;
            continue;
        }
        const double lz = log(fabs(z[i]));
        double s = 0.0;
        for (int k = 0; k < 100000; ++k) {
            const double lt = k * lz - lgamma(a * k + 1.0);
            const double t = exp(lt);
            s += (z[i] < 0.0 && (k & 1)) ? -t : t;
            if (k > 0 && lt < -40.0 && a * k > 2.0) break;
        }
        out[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Nonlinear problem of Section 7: D_t u = (D(u) u_x)_x + c u_x + f on (0, 1)
 * with homogeneous Dirichlet values and a zero initial condition, D(u) =
 * 1 + u^2.  Discretisation: the L1 scheme in time; the diffusion term with
 * the half-point coefficients a_{n+-1/2} = (D(u_{n+-1}) + D(u_n)) / 2; the
 * convection term by upwinding (c > 0 carries information from the right,
 * so u_x is the forward difference).  Solver: the waveform relaxation FAS
 * method with red-black nonlinear Gauss-Seidel (each point's whole time line
 * solved with its neighbours fixed, level by level with Newton's method),
 * full weighting for the residual and the solution, linear interpolation of
 * the coarse correction, V(nu1, nu2) cycles.  1D only; points n = 1..N.
 * D(u) = 1 + q u^2 with q = 1 as in Section 7 (q = 0: the linear problem). */
static double nl_q = 1.0;
static double nl_D(double v) { return 1.0 + nl_q * v * v; }

/* N(u) at every point: (T_M u)_n + stencil terms (the discrete operator). */
static void nl_apply(int N, int M, double h, double cc, const double *r, const double *u, double *out)
{
    for (int m = 0; m < M; ++m)
        for (int n = 1; n <= N; ++n) {
            double s = 0.0;
            for (int j = 0; j <= m; ++j) s += r[m - j] * u[(size_t)j * N + (n - 1)];
            const double *v = u + (size_t)m * N;
            double uc = v[n - 1], ul = at1(v, N, n - 1), ur = at1(v, N, n + 1);
            double ap = 0.5 * (nl_D(ur) + nl_D(uc)), am = 0.5 * (nl_D(ul) + nl_D(uc));
            s -= (ap * (ur - uc) - am * (uc - ul)) / (h * h);
            s -= cc * (ur - uc) / h;
            out[(size_t)m * N + (n - 1)] = s;
        }
}

/* One half-sweep over the points of one colour (0: even n, 1: odd n). */
static void nl_half_sweep(int N, int M, double h, double cc, const double *r, int colour, const double *f, double *u)
{
    for (int n = (colour == 0) ? 2 : 1; n <= N; n += 2) {
        for (int m = 0; m < M; ++m) {
            double hist = 0.0;
            for (int j = 0; j < m; ++j) hist += r[m - j] * u[(size_t)j * N + (n - 1)];
            const double *row = u + (size_t)m * N;
            const double ul = at1(row, N, n - 1), ur = at1(row, N, n + 1), fm = f[(size_t)m * N + (n - 1)];
            double v = row[n - 1];
            for (int it = 0; it < 50; ++it) {
                double ap = 0.5 * (nl_D(ur) + nl_D(v)), am = 0.5 * (nl_D(ul) + nl_D(v));
                double g = r[0] * v + hist - (ap * (ur - v) - am * (v - ul)) / (h * h) - cc * (ur - v) / h - fm;
                double dg = r[0] + (ap + am - nl_q * v * (ur - v) + nl_q * v * (v - ul)) / (h * h) + cc / h;
                double dv = g / dg;
                v -= dv;
                if (fabs(dv) <= 1e-15 * (1.0 + fabs(v))) break;
            }
            u[(size_t)m * N + (n - 1)] = v;
        }
    }
}

static void nl_vcycle(int N, int M, double alpha, double T, double cc, int nu1, int nu2, int first,
                      const double *f, double *u)
{
    double c_unused, *d = (double *)malloc(sizeof(double) * (M + 1)), *r = (double *)malloc(sizeof(double) * M);
    orc_l1_coeffs(M, alpha, T, &c_unused, d, r);
    const double h = 1.0 / (N + 1);
    if (N == 1) {   /* one point: one half-sweep is its exact solve */
        nl_half_sweep(N, M, h, cc, r, 1, f, u);
        free(d); free(r);
        return;
    }
    for (int i = 0; i < nu1; ++i) {
        nl_half_sweep(N, M, h, cc, r, first, f, u);
        nl_half_sweep(N, M, h, cc, r, 1 - first, f, u);
    }
    const int Nc = (N - 1) / 2;
    size_t sf = (size_t)M * N, sc = (size_t)M * Nc;
    double *R = (double *)malloc(sizeof(double) * sf), *uc = (double *)malloc(sizeof(double) * sc);
    double *uc0 = (double *)malloc(sizeof(double) * sc), *fc = (double *)malloc(sizeof(double) * sc);
    double *rc = (double *)malloc(sizeof(double) * sc);
    nl_apply(N, M, h, cc, r, u, R);
    for (size_t i = 0; i < sf; ++i) R[i] = f[i] - R[i];
    orc_restrict(1, N, M, R, rc);
    orc_restrict(1, N, M, u, uc0);
    double *rcoarse = (double *)malloc(sizeof(double) * M);
    orc_l1_coeffs(M, alpha, T, &c_unused, d, rcoarse);
    nl_apply(Nc, M, 1.0 / (Nc + 1), cc, rcoarse, uc0, fc);
    for (size_t i = 0; i < sc; ++i) { fc[i] += rc[i]; uc[i] = uc0[i]; }
    nl_vcycle(Nc, M, alpha, T, cc, nu1, nu2, first, fc, uc);
    for (size_t i = 0; i < sc; ++i) uc[i] -= uc0[i];
    orc_prolong_add(1, Nc, M, uc, u);
    for (int i = 0; i < nu2; ++i) {
        nl_half_sweep(N, M, h, cc, r, first, f, u);
        nl_half_sweep(N, M, h, cc, r, 1 - first, f, u);
    }
    free(R); free(uc); free(uc0); free(fc); free(rc); free(rcoarse); free(d); free(r);
}

/* FAS iteration from u = 0 until the max-norm residual is reduced by tol
 * (Section 7); returns the cycles done, hist[0..its] the residual norms.
 * Not reentrant (q is held in a file-scope variable for the recursion). */
int orc_nl_solve(int N, int M, double alpha, double T, double cc, double q, int nu1, int nu2, int first,
                 double tol, int maxit, const double *f, double *u, double *hist)
{
    nl_q = q;
    size_t sz = (size_t)M * N;
    double c_unused, *d = (double *)malloc(sizeof(double) * (M + 1)), *r = (double *)malloc(sizeof(double) * M);
    orc_l1_coeffs(M, alpha, T, &c_unused, d, r);
    const double h = 1.0 / (N + 1);
    double *R = (double *)malloc(sizeof(double) * sz);
    for (size_t i = 0; i < sz; ++i) u[i] = 0.0;
    double r0 = 0.0;
    int it = 0;
    for (;;) {
        nl_apply(N, M, h, cc, r, u, R);
        double rn = 0.0;
        for (size_t i = 0; i < sz; ++i) rn = fmax(rn, fabs(f[i] - R[i]));
        if (hist) hist[it] = rn;
        if (it == 0) r0 = rn;
        if (rn <= tol * r0 || it >= maxit) break;
        nl_vcycle(N, M, alpha, T, cc, nu1, nu2, first, f, u);
        ++it;
    }
    free(R); free(d); free(r);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Threads the oracle's parallel loops use (for reporting its timings).     */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
