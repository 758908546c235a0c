// Host runtime and C ABI of the MGWR solver (include/mgwr.h).
//
// Method: Gaspar & Rodrigo, "Multigrid waveform relaxation for the
// time-fractional heat equation", arXiv:1608.05400.  The L1 discretisation
// (Section 2) makes the space-time matrix T_M (x) I + A_h with T_M lower
// triangular Toeplitz (Section 5).  Algorithm 1 (Section 3) is run with
//   * smoother: red-black waveform relaxation; one half-sweep solves
//     (T_M + sigma I) x = b for every point of a colour.  The inverse of a
//     lower-triangular Toeplitz matrix is lower-triangular Toeplitz and its
//     first column can be computed once (Section 5.2), so a half-sweep is one
//     causal Toeplitz product of that column with the colour's right-hand
//     sides (an MFMA GEMM over all points of the colour);
//   * defect: one causal Toeplitz product with T_M plus the stencil, fused;
//   * full weighting / linear (bilinear) interpolation, coarsening in space
//     only down to one point, where one sweep is the exact line solve.
// mgwr_solve runs either Algorithm 1 on u directly (MGWR_FP64), or an outer
// iterative refinement whose residual is FP64 with the iterate carried as a
// double-double (hi in the caller's u, lo internal) and whose correction
// comes from one cycle on the error equation in FP64, FP32 or split-BF16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "mgwr.h"
#include "mgwr_internal.h"

using namespace mgwr;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(e_ == hipErrorOutOfMemory ? MGWR_ENOMEM : MGWR_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
    } while (0)

#define CHK(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ < 0) return rc_;   \
    } while (0)

// Split-BF16 products are used only where a launch has at least this many
// columns; narrower levels (the coarse grids) run their products in FP32.
constexpr int kBf16MinCols = 128;

// ---------------------------------------------------------------------------
// L1 weights (Section 2, L1 scheme; Section 5, r_i).  d_k for k >= 2 as
// -k^b expm1(b log1p(-1/k)); the second difference d_i - d_{i-1} for large i
// from the binomial series of (1 + e)^b + (1 - e)^b - 2, e = 1/(i-1), so that
// no digits are lost to cancellation.
double l1_d(long k, double b)
{
    if (k <= 0) return 0.0;
    if (k == 1) return 1.0;
    double x = (double)k;
    return -std::pow(x, b) * std::expm1(b * std::log1p(-1.0 / x));
}

double l1_second_diff(long i, double b)   // d_i - d_{i-1}, i >= 2
{
    if (i == 2) return std::pow(2.0, b) - 2.0;
    double x = (double)(i - 1);
    if (x < 4.0) {
        double A = std::expm1(b * std::log1p(1.0 / x));
        double B = std::expm1(b * std::log1p(-1.0 / x));
        return std::pow(x, b) * (A + B);
    }
    double eps2 = 1.0 / (x * x), term = 1.0, sum = 0.0, binom = 1.0;
    for (int k = 1; k <= 60; ++k) {
        binom *= (b - (k - 1)) / k;          // C(b, k)
        if (k % 2 == 0) {
            term *= eps2;
            double t = binom * term;
            sum += t;
            if (std::fabs(t) <= 1e-18 * std::fabs(sum)) break;
        }
    }
    return std::pow(x, b) * 2.0 * sum;
}

void l1_weights(int M, double alpha, double T, double &c, std::vector<double> &r,
                std::vector<double> &d)
{
    double b = 1.0 - alpha, tau = T / M;
    c = std::pow(tau, -alpha) / std::tgamma(2.0 - alpha);
    r.assign(M, 0.0);
    d.assign(M + 1, 0.0);
    for (long k = 1; k <= M; ++k) d[k] = l1_d(k, b);
    r[0] = c;
    for (long i = 2; i <= M; ++i) r[i - 1] = c * l1_second_diff(i, b);
}

// First column of (T_M + sigma I)^{-1} by forward substitution.  T_M + sigma I
// is lower triangular with positive diagonal and non-positive off-diagonal
// entries, so every term of the recurrence is non-negative (no cancellation).
void inverse_column(const std::vector<double> &r, double sigma, std::vector<double> &lam)
{
    const int M = (int)r.size();
    lam.assign(M, 0.0);
    const double dinv = 1.0 / (r[0] + sigma);
    lam[0] = dinv;
    for (int m = 1; m < M; ++m) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int k = 1;
        for (; k + 3 <= m; k += 4) {
            s0 -= r[k] * lam[m - k];
            s1 -= r[k + 1] * lam[m - k - 1];
            s2 -= r[k + 2] * lam[m - k - 2];
            s3 -= r[k + 3] * lam[m - k - 3];
        }
        for (; k <= m; ++k) s0 -= r[k] * lam[m - k];
        lam[m] = ((s0 + s1) + (s2 + s3)) * dinv;
    }
}

// ---------------------------------------------------------------------------
struct Level {
    int n = 0;
    long P = 0;
    int Pc[2] = {0, 0};
    double h = 0, ih2 = 0, sigma = 0;
    ToepCoef inv;     // first column of (T_M + sigma I)^{-1}
    ToepCoef inv_h;   // the same without its first entry (history part)
    double lam0 = 0;  // first entry of that column
    double *u64 = nullptr, *f64 = nullptr;  // FP64 hierarchy (levels below the finest)
    double *e = nullptr, *fe = nullptr;     // inner hierarchy of the refinement (all levels)
};

}  // namespace

struct mgwr_ctx {
    int N = 0, M = 0, dims = 1;
    double alpha = 0, T = 1;
    mgwr_options opt{};
    hipStream_t stream = nullptr;
    int device = 0;
    double c = 0;
    std::vector<double> r_host, d_host;
    ToepCoef tm;      // first column of T_M
    ToepCoef tm_h;    // the same without r_1 (history part)
    double *cd = nullptr;
    std::vector<Level> lv;
    int Mpad = 0;
    long maxPc = 0;
    // workspace
    double *res64 = nullptr, *panel64 = nullptr, *ulo = nullptr, *rs64 = nullptr;
    float *panel32 = nullptr, *op32 = nullptr;
    uint16_t *pk_hi = nullptr, *pk_lo = nullptr;
    long pk_ld = 0;
    double *partials = nullptr, *norms_dev = nullptr, *norms_host = nullptr;
    void *part = nullptr;            // split-K partials of the Toeplitz products
    size_t part_cap = 0;
    // per-launch timing of the Toeplitz products
    bool prof = false;
    struct Pending { hipEvent_t a, b; mgwr_kernel_record rec; };
    std::vector<Pending> pending;
    std::vector<mgwr_kernel_record> records;
    std::vector<hipEvent_t> event_pool;
    int inner_prec = -1;             // precision the inner buffers exist for
    std::vector<void *> inner_alloc; // buffers owned by the inner hierarchy
    std::vector<void *> alloc;       // everything else
};

namespace {

int dmalloc(mgwr_ctx *h, std::vector<void *> &list, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? MGWR_ENOMEM : MGWR_EDEVICE,
                    "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    list.push_back(*p);
    (void)h;
    return MGWR_OK;
}

void free_list(std::vector<void *> &list)
{
    for (void *p : list) hipFree(p);
    list.clear();
}

int upload_coef(mgwr_ctx *h, ToepCoef &c, const std::vector<double> &v)
{
    c.n = (int)v.size();
    c.nq = (c.n + 15) / 16 + 4 * kQOff;
    CHK(dmalloc(h, h->alloc, (void **)&c.d64, sizeof(double) * c.n));
    CHK(dmalloc(h, h->alloc, (void **)&c.d32, sizeof(float) * c.n));
    CHK(dmalloc(h, h->alloc, (void **)&c.fhi, sizeof(uint16_t) * 512 * (size_t)c.nq));
    CHK(dmalloc(h, h->alloc, (void **)&c.flo, sizeof(uint16_t) * 512 * (size_t)c.nq));
    HIPCHK(hipMemcpy(c.d64, v.data(), sizeof(double) * c.n, hipMemcpyHostToDevice));
    HIPCHK(launch_build_coef(c, nullptr));
    return MGWR_OK;
}

// Multiply-adds of a Toeplitz product that are not structurally zero.
double product_flops(const GemmArgs &a)
{
    double macs = 0;
    for (int i = 0; i < a.M; ++i) {
        long lo = std::max(0, a.off + i - a.coef->n + 1), hi = std::min(a.K - 1, i + a.off);
        if (hi >= lo) macs += (double)(hi - lo + 1);
    }
    return 2.0 * macs * a.P;
}

int kernel_id(const GemmArgs &a)
{
    int narrow = (a.mode != GM_BF16X3 && a.P <= 32) ? 1 : 0;
    return (a.mode << 4) | (a.epi << 1) | narrow;
}

hipEvent_t take_event(mgwr_ctx *h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int resolve_profile(mgwr_ctx *h)
{
    if (h->pending.empty()) return MGWR_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (auto &p : h->pending) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        p.rec.ms = ms;
        h->records.push_back(p.rec);
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    return MGWR_OK;
}

int run_gemm(mgwr_ctx *h, const GemmArgs &a_in, int level)
{
    GemmArgs a = a_in;
    a.part = h->part;
    a.part_cap = h->part_cap;
    if (!h->prof) {
        HIPCHK(launch_toep_gemm(a, h->stream));
        return MGWR_OK;
    }
    mgwr_ctx::Pending p;
    p.a = take_event(h);
    p.b = take_event(h);
    if (!p.a || !p.b) return fail(MGWR_EDEVICE, "hipEventCreate failed");
    p.rec.kernel = kernel_id(a); p.rec.level = level; p.rec.M = a.M; p.rec.P = a.P; p.rec.K = a.K;
    p.rec.flops = product_flops(a); p.rec.ms = 0;
    HIPCHK(hipEventRecord(p.a, h->stream));
    HIPCHK(launch_toep_gemm(a, h->stream));
    HIPCHK(hipEventRecord(p.b, h->stream));
    h->pending.push_back(p);
    if (h->pending.size() >= 4096) CHK(resolve_profile(h));
    return MGWR_OK;
}

bool is_pow2m1(int N)
{
    return N >= 1 && ((N + 1) & N) == 0;
}

int check_opts(const mgwr_options *o)
{
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 16 || o->nu2 > 16)
        return fail(MGWR_EINVAL, "nu1, nu2 must be in [0, 16] with nu1 + nu2 >= 1");
    if (o->gamma < 1 || o->gamma > 2) return fail(MGWR_EINVAL, "gamma must be 1 (V) or 2 (W)");
    if (o->maxit < 0) return fail(MGWR_EINVAL, "maxit must be >= 0");
    if (o->norm != MGWR_NORM_MAX && o->norm != MGWR_NORM_L2) return fail(MGWR_EINVAL, "bad norm");
    if (o->precision < MGWR_FP64 || o->precision > MGWR_FP64_REFINED)
        return fail(MGWR_EINVAL, "bad precision");
    if (o->first_colour != 0 && o->first_colour != 1) return fail(MGWR_EINVAL, "first_colour must be 0 or 1");
    if (o->smoother != MGWR_SMOOTH_INVERSE && o->smoother != MGWR_SMOOTH_DC)
        return fail(MGWR_EINVAL, "bad smoother");
    if (o->smoother == MGWR_SMOOTH_DC)
        return fail(MGWR_EINVAL, "divide-and-conquer smoother is not available in this build");
    if (!(o->L > 0) || !std::isfinite(o->L)) return fail(MGWR_EINVAL, "L must be positive");
    if (!(o->stall >= 0) || o->stall >= 1.0) return fail(MGWR_EINVAL, "stall must be in [0, 1)");
    return MGWR_OK;
}

// Allocate the buffers the refinement with precision `prec` needs.  The
// inner hierarchy is FP64 in every precision; FP32 / split-BF16 appear only
// as product operands.
int alloc_inner(mgwr_t h, int prec)
{
    if (h->inner_prec == prec) return MGWR_OK;
    free_list(h->inner_alloc);
    for (auto &L : h->lv) { L.e = nullptr; L.fe = nullptr; }
    h->rs64 = nullptr; h->panel32 = nullptr; h->op32 = nullptr;
    h->pk_hi = h->pk_lo = nullptr;
    h->inner_prec = -1;
    const long M = h->M;
    const int nl = (int)h->lv.size();
    const long Pf = h->lv.back().P;
    if (prec != MGWR_FP64) {
        for (int l = 0; l < nl; ++l) {
            CHK(dmalloc(h, h->inner_alloc, (void **)&h->lv[l].e, sizeof(double) * M * h->lv[l].P));
            if (l < nl - 1)
                CHK(dmalloc(h, h->inner_alloc, (void **)&h->lv[l].fe, sizeof(double) * M * h->lv[l].P));
        }
        h->lv.back().fe = h->res64;   // the outer residual is the finest right-hand side
        CHK(dmalloc(h, h->inner_alloc, (void **)&h->rs64, sizeof(double) * M * Pf));
    }
    if (prec == MGWR_MIXED_FP32 || prec == MGWR_MIXED_BF16X3) {
        CHK(dmalloc(h, h->inner_alloc, (void **)&h->panel32, sizeof(float) * M * h->maxPc));
        CHK(dmalloc(h, h->inner_alloc, (void **)&h->op32, sizeof(float) * M * Pf));
    }
    if (prec == MGWR_MIXED_BF16X3) {
        h->pk_ld = (Pf + 127) / 128 * 128;
        size_t bytes = sizeof(uint16_t) * (size_t)h->Mpad * h->pk_ld;
        CHK(dmalloc(h, h->inner_alloc, (void **)&h->pk_hi, bytes));
        CHK(dmalloc(h, h->inner_alloc, (void **)&h->pk_lo, bytes));
    }
    h->inner_prec = prec;
    return MGWR_OK;
}

// ---------------------------------------------------------------------------
// One cycle over a hierarchy whose per-level iterate/rhs are given (FP64).
struct Hier {
    int prec;                     // precision of the products (enum mgwr_precision)
    std::vector<double *> u, f;   // per level
    const double *g;              // initial condition on the finest level (plain FP64 only)
    double *rscratch;             // residual scratch [M][P_fine]
};

int level_mode(const Hier &H, long cols)
{
    if (H.prec == MGWR_FP64 || H.prec == MGWR_FP64_REFINED) return GM_F64;
    if (H.prec == MGWR_MIXED_BF16X3 && cols >= kBf16MinCols) return GM_BF16X3;
    return GM_F32;
}

// One half-sweep: every point of `colour` on level `lev` gets the solution of
// (T_M + sigma I) x = b along its time line, as one Toeplitz product with the
// precomputed inverse column.  In FP64 the product is the whole solve; in
// FP32 / split-BF16 the right-hand-side kernel writes lambda_0 b (FP64) into
// the colour's points and the product adds the strictly lower (history) part.
int half_sweep(mgwr_t h, const Hier &H, int lev, int colour)
{
    Level &L = h->lv[lev];
    const int Pc = L.Pc[colour];
    if (Pc == 0) return MGWR_OK;
    const bool fine = (lev == (int)h->lv.size() - 1);
    const double *g = fine ? H.g : nullptr;
    GemmArgs a;
    a.mode = level_mode(H, Pc);
    a.M = h->M; a.P = Pc; a.K = h->M; a.off = 0;
    a.ea.out = H.u[lev]; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n; a.ea.colour = colour;
    if (a.mode == GM_F64) {
        HIPCHK(launch_rhs_panel(0, h->dims, L.n, colour, h->M, h->Mpad, H.f[lev], H.u[lev], h->cd, g, L.ih2,
                                0.0, h->panel64, nullptr, Pc, h->stream));
        a.coef = &L.inv; a.epi = EPI_SCATTER; a.B = h->panel64; a.ldb = Pc;
    } else if (a.mode == GM_F32) {
        HIPCHK(launch_rhs_panel(1, h->dims, L.n, colour, h->M, h->Mpad, H.f[lev], H.u[lev], h->cd, g, L.ih2,
                                L.lam0, h->panel32, nullptr, Pc, h->stream));
        a.coef = &L.inv_h; a.epi = EPI_SCATTER_ADD; a.B = h->panel32; a.ldb = Pc;
    } else {
        long ldp = (Pc + 127) / 128 * 128;
        HIPCHK(launch_rhs_panel(2, h->dims, L.n, colour, h->M, h->Mpad, H.f[lev], H.u[lev], h->cd, g, L.ih2,
                                L.lam0, h->pk_hi, h->pk_lo, ldp, h->stream));
        a.coef = &L.inv_h; a.epi = EPI_SCATTER_ADD; a.Bhi = h->pk_hi; a.Blo = h->pk_lo; a.ldb = ldp;
    }
    CHK(run_gemm(h, a, lev));
    return MGWR_OK;
}

int sweep(mgwr_t h, const Hier &H, int lev)
{
    const int c0 = h->opt.first_colour;
    CHK(half_sweep(h, H, lev, c0));
    CHK(half_sweep(h, H, lev, 1 - c0));
    return MGWR_OK;
}

// out = f + c d g - T_M u - A_h u on level lev: the Toeplitz product (all
// of T_M u in FP64, its history part otherwise) stored into out, then the
// stencil part and the diagonal r_1 u applied by a bandwidth kernel.
int level_residual(mgwr_t h, const Hier &H, int lev, double *out)
{
    Level &L = h->lv[lev];
    const bool fine = (lev == (int)h->lv.size() - 1);
    GemmArgs a;
    a.mode = level_mode(H, L.P);
    a.M = h->M; a.P = (int)L.P; a.K = h->M; a.off = 0;
    a.epi = EPI_STORE;
    a.ea.out = out; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n;
    const double diag = (a.mode == GM_F64) ? 0.0 : h->c;
    if (a.mode == GM_F64) {
        a.coef = &h->tm; a.B = H.u[lev]; a.ldb = L.P;
    } else if (a.mode == GM_F32) {
        HIPCHK(launch_operand(1, h->M, h->Mpad, (int)L.P, H.u[lev], h->op32, nullptr, L.P, h->stream));
        a.coef = &h->tm_h; a.B = h->op32; a.ldb = L.P;
    } else {
        long ldp = (L.P + 127) / 128 * 128;
        HIPCHK(launch_operand(2, h->M, h->Mpad, (int)L.P, H.u[lev], h->pk_hi, h->pk_lo, ldp, h->stream));
        a.coef = &h->tm_h; a.Bhi = h->pk_hi; a.Blo = h->pk_lo; a.ldb = ldp;
    }
    CHK(run_gemm(h, a, lev));
    HIPCHK(launch_resid_post(h->dims, L.n, h->M, H.f[lev], H.u[lev], nullptr, h->cd, fine ? H.g : nullptr,
                             L.ih2, diag, out, h->stream));
    return MGWR_OK;
}

int cycle(mgwr_t h, const Hier &H, int lev)
{
    const mgwr_options &o = h->opt;
    if (lev == 0) return sweep(h, H, 0);
    for (int i = 0; i < o.nu1; ++i) CHK(sweep(h, H, lev));
    Level &L = h->lv[lev];
    CHK(level_residual(h, H, lev, H.rscratch));
    HIPCHK(launch_restrict(h->dims, L.n, h->M, H.rscratch, H.f[lev - 1], h->stream));
    HIPCHK(launch_fill(h->M, h->lv[lev - 1].P, nullptr, H.u[lev - 1], h->stream));
    for (int k = 0; k < o.gamma; ++k) CHK(cycle(h, H, lev - 1));
    HIPCHK(launch_prolong_add(h->dims, h->lv[lev - 1].n, h->M, H.u[lev - 1], H.u[lev], h->stream));
    for (int i = 0; i < o.nu2; ++i) CHK(sweep(h, H, lev));
    return MGWR_OK;
}

Hier plain_hier(mgwr_t h, const double *f, const double *g, double *u)
{
    Hier H;
    H.prec = MGWR_FP64; H.g = g; H.rscratch = h->res64;
    for (auto &L : h->lv) { H.u.push_back(L.u64); H.f.push_back(L.f64); }
    H.u.back() = u; H.f.back() = (double *)f;
    return H;
}

Hier inner_hier(mgwr_t h)
{
    Hier H;
    H.prec = h->opt.precision; H.g = nullptr; H.rscratch = h->rs64;
    for (auto &L : h->lv) { H.u.push_back(L.e); H.f.push_back(L.fe); }
    return H;
}

// FP64 residual of the finest level into res (double-double iterate when lo
// != nullptr) and its norms (host, synchronising).
// cold: u is the initial iterate g at every time level (lo zero).  Then
// T_M u = c d_m g exactly (the rows of T_M sum to c d_m), so the product is
// replaced by writing c d_m g.
int fine_residual_norms(mgwr_t h, const double *f, const double *g, const double *u, const double *lo,
                        double *res, double norms[2], bool cold = false)
{
    Level &L = h->lv.back();
    if (cold) {
        HIPCHK(launch_scaled_fill(h->M, L.P, h->cd, g, res, h->stream));
    } else {
        GemmArgs a;
        a.mode = GM_F64;
        a.M = h->M; a.P = (int)L.P; a.K = h->M; a.off = 0; a.coef = &h->tm;
        a.epi = EPI_STORE;
        a.ea.out = res; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n;
        a.B = u; a.ldb = L.P;
        CHK(run_gemm(h, a, (int)h->lv.size() - 1));
    }
    HIPCHK(launch_resid_post(h->dims, L.n, h->M, f, u, lo, h->cd, g, L.ih2, 0.0, res, h->stream));
    if (norms) {
        int nblk = 0;
        HIPCHK(launch_norm_partials((long)h->M * L.P, res, h->partials, &nblk, h->stream));
        HIPCHK(launch_norm_final(nblk, h->partials, h->norms_dev, h->stream));
        HIPCHK(hipMemcpyAsync(h->norms_host, h->norms_dev, 2 * sizeof(double), hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        norms[0] = h->norms_host[0];
        norms[1] = h->norms_host[1];
    }
    return MGWR_OK;
}

int check_ptr(const void *p, const char *name)
{
    if (!p) return fail(MGWR_EINVAL, "%s must not be NULL", name);
    if (((uintptr_t)p) % 8 != 0) return fail(MGWR_EINVAL, "%s must be 8-byte aligned", name);
    return MGWR_OK;
}

int set_device(mgwr_t h)
{
    HIPCHK(hipSetDevice(h->device));
    return MGWR_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *mgwr_last_error(void) { return g_err.c_str(); }

int mgwr_default_options(mgwr_options *o)
{
    if (!o) return fail(MGWR_EINVAL, "options pointer is NULL");
    memset(o, 0, sizeof *o);
    o->nu1 = 1; o->nu2 = 1; o->gamma = 1; o->maxit = 100; o->norm = MGWR_NORM_MAX;
    o->warm_start = 0; o->precision = MGWR_FP64; o->first_colour = 0;
    o->smoother = MGWR_SMOOTH_INVERSE; o->dc_block = 0; o->L = 1.0; o->stall = 0.5;
    return MGWR_OK;
}

int mgwr_l1_weights(int M, double alpha, double T, double *c, double *r)
{
    if (M < 1) return fail(MGWR_EINVAL, "M must be >= 1");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(MGWR_EINVAL, "alpha must be in (0, 1]");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(MGWR_EINVAL, "T must be positive");
    if (!c || !r) return fail(MGWR_EINVAL, "output pointers must not be NULL");
    std::vector<double> rv, dv;
    l1_weights(M, alpha, T, *c, rv, dv);
    memcpy(r, rv.data(), sizeof(double) * M);
    return MGWR_OK;
}

int mgwr_create(int N, int M, double alpha, double T, int dims, mgwr_t *out)
{
    return mgwr_create_ex(N, M, alpha, T, dims, nullptr, out);
}

int mgwr_destroy(mgwr_t h)
{
    if (!h) return MGWR_OK;
    hipSetDevice(h->device);
    if (h->stream) hipStreamSynchronize(h->stream);
    free_list(h->inner_alloc);
    free_list(h->alloc);
    if (h->norms_host) hipHostFree(h->norms_host);
    for (auto &p : h->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
    for (auto e : h->event_pool) hipEventDestroy(e);
    delete h;
    return MGWR_OK;
}

int mgwr_create_ex(int N, int M, double alpha, double T, int dims, const mgwr_options *opts, mgwr_t *out)
{
    if (!out) return fail(MGWR_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (dims != 1 && dims != 2) return fail(MGWR_EINVAL, "dims must be 1 or 2 (got %d)", dims);
    if (!is_pow2m1(N) || N > (dims == 1 ? (1 << 24) - 1 : (1 << 14) - 1))
        return fail(MGWR_EINVAL, "N must be 2^k - 1 (got %d)", N);
    if (M < 1 || M > (1 << 22)) return fail(MGWR_EINVAL, "M must be in [1, 2^22] (got %d)", M);
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(MGWR_EINVAL, "alpha must be in (0, 1] (got %g)", alpha);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(MGWR_EINVAL, "T must be positive and finite");
    mgwr_options o;
    mgwr_default_options(&o);
    if (opts) o = *opts;
    CHK(check_opts(&o));

    mgwr_ctx *h = new mgwr_ctx();
    h->N = N; h->M = M; h->dims = dims; h->alpha = alpha; h->T = T; h->opt = o;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(MGWR_EDEVICE, "no HIP device available");
    }
    int rc = [&]() -> int {
        l1_weights(M, alpha, T, h->c, h->r_host, h->d_host);
        h->Mpad = (M + 127) / 128 * 128;
        // levels: finest n = N, then (n - 1) / 2 down to 1
        std::vector<int> ns;
        for (int n = N; n >= 1; n = (n - 1) / 2) {
            ns.push_back(n);
            if (n == 1) break;
        }
        std::reverse(ns.begin(), ns.end());
        h->lv.resize(ns.size());
        for (size_t l = 0; l < ns.size(); ++l) {
            Level &L = h->lv[l];
            L.n = ns[l];
            L.P = (dims == 1) ? L.n : (long)L.n * L.n;
            L.Pc[0] = colour_count(dims, L.n, 0);
            L.Pc[1] = colour_count(dims, L.n, 1);
            L.h = o.L / (L.n + 1);
            L.ih2 = 1.0 / (L.h * L.h);
            L.sigma = (dims == 1 ? 2.0 : 4.0) * L.ih2;
            h->maxPc = std::max<long>(h->maxPc, std::max(L.Pc[0], L.Pc[1]));
        }
        // inverse columns, one host thread per level
        std::vector<std::vector<double>> lam(h->lv.size());
        std::vector<std::thread> th;
        for (size_t l = 0; l < h->lv.size(); ++l)
            th.emplace_back([&, l]() { inverse_column(h->r_host, h->lv[l].sigma, lam[l]); });
        for (auto &t : th) t.join();
        CHK(upload_coef(h, h->tm, h->r_host));
        std::vector<double> hist = h->r_host;
        hist[0] = 0.0;
        CHK(upload_coef(h, h->tm_h, hist));
        for (size_t l = 0; l < h->lv.size(); ++l) {
            CHK(upload_coef(h, h->lv[l].inv, lam[l]));
            h->lv[l].lam0 = lam[l][0];
            lam[l][0] = 0.0;
            CHK(upload_coef(h, h->lv[l].inv_h, lam[l]));
        }
        std::vector<double> cdv(M);
        for (int m = 0; m < M; ++m) cdv[m] = h->c * h->d_host[m + 1];
        CHK(dmalloc(h, h->alloc, (void **)&h->cd, sizeof(double) * M));
        HIPCHK(hipMemcpy(h->cd, cdv.data(), sizeof(double) * M, hipMemcpyHostToDevice));
        const long Pf = h->lv.back().P;
        for (size_t l = 0; l + 1 < h->lv.size(); ++l) {
            CHK(dmalloc(h, h->alloc, (void **)&h->lv[l].u64, sizeof(double) * M * h->lv[l].P));
            CHK(dmalloc(h, h->alloc, (void **)&h->lv[l].f64, sizeof(double) * M * h->lv[l].P));
        }
        CHK(dmalloc(h, h->alloc, (void **)&h->res64, sizeof(double) * M * Pf));
        CHK(dmalloc(h, h->alloc, (void **)&h->panel64, sizeof(double) * M * h->maxPc));
        CHK(dmalloc(h, h->alloc, (void **)&h->ulo, sizeof(double) * M * Pf));
        CHK(dmalloc(h, h->alloc, (void **)&h->partials, sizeof(double) * 2 * 2048));
        // split-K scratch: the largest any product of this hierarchy needs
        size_t part = 0;
        for (const Level &L : h->lv)
            for (int mode = GM_F64; mode <= GM_BF16X3; ++mode) {
                long cols[3] = {L.Pc[0], L.Pc[1], L.P};
                for (long P : cols)
                    if (P > 0) part = std::max(part, splitk_bytes(mode, M, (int)P, M, 0, M));
            }
        if (part > 0) {
            CHK(dmalloc(h, h->alloc, &h->part, part));
            h->part_cap = part;
        }
        CHK(dmalloc(h, h->alloc, (void **)&h->norms_dev, sizeof(double) * 2));
        HIPCHK(hipHostMalloc((void **)&h->norms_host, 2 * sizeof(double), hipHostMallocDefault));
        CHK(alloc_inner(h, o.precision));
        HIPCHK(hipDeviceSynchronize());
        return MGWR_OK;
    }();
    if (rc < 0) {
        std::string msg = g_err;
        mgwr_destroy(h);
        g_err = msg;
        return rc;
    }
    *out = h;
    return MGWR_OK;
}

int mgwr_set_options(mgwr_t h, const mgwr_options *opts)
{
    if (!h || !opts) return fail(MGWR_EINVAL, "NULL argument");
    CHK(check_opts(opts));
    if (opts->L != h->opt.L) return fail(MGWR_EINVAL, "L is fixed at creation (use mgwr_create_ex)");
    CHK(set_device(h));
    CHK(alloc_inner(h, opts->precision));
    h->opt = *opts;
    return MGWR_OK;
}

int mgwr_get_options(mgwr_t h, mgwr_options *opts)
{
    if (!h || !opts) return fail(MGWR_EINVAL, "NULL argument");
    *opts = h->opt;
    return MGWR_OK;
}

int mgwr_set_stream(mgwr_t h, void *hip_stream)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    h->stream = (hipStream_t)hip_stream;
    return MGWR_OK;
}

int mgwr_levels(mgwr_t h)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    return (int)h->lv.size();
}

int mgwr_get_column(mgwr_t h, int which, double *out)
{
    if (!h || !out) return fail(MGWR_EINVAL, "NULL argument");
    if (which < -1 || which >= (int)h->lv.size()) return fail(MGWR_EINVAL, "bad level %d", which);
    CHK(set_device(h));
    const ToepCoef &c = which < 0 ? h->tm : h->lv[which].inv;
    HIPCHK(hipMemcpy(out, c.d64, sizeof(double) * c.n, hipMemcpyDeviceToHost));
    return MGWR_OK;
}

int mgwr_smooth(mgwr_t h, const double *f, const double *g, double *u, int sweeps)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    if (sweeps < 0) return fail(MGWR_EINVAL, "sweeps must be >= 0");
    CHK(set_device(h));
    Hier H = plain_hier(h, f, g, u);
    for (int s = 0; s < sweeps; ++s) CHK(sweep(h, H, (int)h->lv.size() - 1));
    return MGWR_OK;
}

int mgwr_residual(mgwr_t h, const double *f, const double *g, const double *u, double *r, double *norms)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    CHK(check_ptr(r, "r"));
    CHK(set_device(h));
    double nrm[2];
    CHK(fine_residual_norms(h, f, g, u, nullptr, r, norms ? nrm : nullptr));
    if (norms) { norms[0] = nrm[0]; norms[1] = nrm[1]; }
    return MGWR_OK;
}

int mgwr_vcycle(mgwr_t h, const double *f, const double *g, double *u)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    CHK(set_device(h));
    Hier H = plain_hier(h, f, g, u);
    return cycle(h, H, (int)h->lv.size() - 1);
}

int mgwr_solve(mgwr_t h, const double *f, const double *g, double *u, double tol, mgwr_info *info)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    if (!(tol >= 0.0)) return fail(MGWR_EINVAL, "tol must be >= 0");
    CHK(set_device(h));
    const mgwr_options &o = h->opt;
    const int prec = o.precision;
    const bool refine = prec != MGWR_FP64;
    CHK(alloc_inner(h, prec));
    const long Pf = h->lv.back().P;
    const long n = (long)h->M * Pf;
    if (!o.warm_start) HIPCHK(launch_fill(h->M, Pf, g, u, h->stream));
    if (refine) HIPCHK(hipMemsetAsync(h->ulo, 0, sizeof(double) * n, h->stream));
    Hier Hp = plain_hier(h, f, g, u);
    Hier Hi;
    if (refine) Hi = inner_hier(h);

    mgwr_info inf;
    memset(&inf, 0, sizeof inf);
    int status = MGWR_NOT_CONVERGED;
    double r0 = 0, prev = 0, rn = 0;
    int it = 0, slow = 0;
    for (;; ++it) {
        double nrm[2];
        CHK(fine_residual_norms(h, f, g, u, refine ? h->ulo : nullptr, h->res64, nrm,
                                it == 0 && !o.warm_start));
        rn = nrm[o.norm];
        if (!std::isfinite(nrm[1]) || !std::isfinite(rn)) {
            status = MGWR_ENONFINITE;
            fail(MGWR_ENONFINITE, "non-finite residual after %d cycles", it);
            break;
        }
        if (it < 128) inf.hist[it] = rn;
        if (it == 0) r0 = rn;
        if (rn <= tol * r0) { status = MGWR_OK; break; }
        if (it > 0 && rn > 1e6 * r0) {
            status = MGWR_EDIVERGED;
            fail(MGWR_EDIVERGED, "residual grew from %g to %g", r0, rn);
            break;
        }
        // Stagnation: a cycle that does not reduce the residual by the factor
        // `stall`.  Near the rounding floor (below 1e-6 r0) one such cycle
        // ends the solve; above it three in a row do (a refinement step may
        // raise the residual once while it removes the smooth error).
        if (it > 0 && o.stall > 0 && rn > o.stall * prev) {
            ++slow;
            if (rn < 1e-6 * r0 || slow >= 3) { status = MGWR_STAGNATED; break; }
        } else {
            slow = 0;
        }
        if (it >= o.maxit) { status = MGWR_NOT_CONVERGED; break; }
        prev = rn;
        if (!refine) {
            CHK(cycle(h, Hp, (int)h->lv.size() - 1));
        } else {
            Level &L = h->lv.back();
            HIPCHK(launch_fill(h->M, L.P, nullptr, L.e, h->stream));
            CHK(cycle(h, Hi, (int)h->lv.size() - 1));
            HIPCHK(launch_dd_update(n, L.e, u, h->ulo, h->stream));
        }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    inf.iters = it;
    inf.status = status;
    inf.r0 = r0;
    inf.rk = rn;
    inf.relres = r0 > 0 ? rn / r0 : 0.0;
    inf.mean_factor = (it > 0 && r0 > 0) ? std::pow(rn / r0, 1.0 / it) : 0.0;
    if (info) *info = inf;
    return status;
}

int mgwr_toeplitz_apply(mgwr_t h, int which, int precision, const double *B, int ldb, int P, double *C,
                        int ldc)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(B, "B"));
    CHK(check_ptr(C, "C"));
    if (which < -1 || which >= (int)h->lv.size()) return fail(MGWR_EINVAL, "bad level %d", which);
    if (P < 1 || ldb < P || ldc < P) return fail(MGWR_EINVAL, "need 1 <= P <= ldb, ldc");
    if (precision < MGWR_FP64 || precision > MGWR_FP64_REFINED) return fail(MGWR_EINVAL, "bad precision");
    CHK(set_device(h));
    const ToepCoef *coef = which < 0 ? &h->tm : &h->lv[which].inv;
    GemmArgs a;
    a.M = h->M; a.P = P; a.K = h->M; a.off = 0; a.coef = coef; a.epi = EPI_STORE;
    a.ea.out = C; a.ea.ldo = ldc;
    if (precision == MGWR_FP64 || precision == MGWR_FP64_REFINED) {
        a.mode = GM_F64; a.B = B; a.ldb = ldb;
        CHK(run_gemm(h, a, which));
        return MGWR_OK;
    }
    // FP32 / split-BF16 operands are built from a contiguous FP64 copy (test
    // path; allocates temporaries)
    std::vector<void *> tmp;
    long n = (long)h->M * P;
    int rc = [&]() -> int {
        double *bd = nullptr;
        CHK(dmalloc(h, tmp, (void **)&bd, sizeof(double) * n));
        HIPCHK(hipMemcpy2DAsync(bd, sizeof(double) * P, B, sizeof(double) * ldb, sizeof(double) * P, h->M,
                                hipMemcpyDeviceToDevice, h->stream));
        if (precision == MGWR_MIXED_FP32) {
            float *b32 = nullptr;
            CHK(dmalloc(h, tmp, (void **)&b32, sizeof(float) * n));
            HIPCHK(launch_operand(1, h->M, h->Mpad, P, bd, b32, nullptr, P, h->stream));
            a.mode = GM_F32; a.B = b32; a.ldb = P;
        } else {
            long ldp = (P + 127) / 128 * 128;
            uint16_t *hi = nullptr, *lo = nullptr;
            size_t bytes = sizeof(uint16_t) * (size_t)h->Mpad * ldp;
            CHK(dmalloc(h, tmp, (void **)&hi, bytes));
            CHK(dmalloc(h, tmp, (void **)&lo, bytes));
            HIPCHK(launch_operand(2, h->M, h->Mpad, P, bd, hi, lo, ldp, h->stream));
            a.mode = GM_BF16X3; a.Bhi = hi; a.Blo = lo; a.ldb = ldp;
        }
        CHK(run_gemm(h, a, which));
        return MGWR_OK;
    }();
    hipStreamSynchronize(h->stream);
    free_list(tmp);
    return rc;
}

int mgwr_profile_enable(mgwr_t h, int on)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(set_device(h));
    CHK(resolve_profile(h));
    if (on) h->records.clear();
    h->prof = on != 0;
    return MGWR_OK;
}

int mgwr_profile_count(mgwr_t h)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(set_device(h));
    CHK(resolve_profile(h));
    return (int)h->records.size();
}

int mgwr_profile_get(mgwr_t h, int i, mgwr_kernel_record *rec)
{
    if (!h || !rec) return fail(MGWR_EINVAL, "NULL argument");
    CHK(resolve_profile(h));
    if (i < 0 || i >= (int)h->records.size()) return fail(MGWR_EINVAL, "record %d out of range", i);
    *rec = h->records[i];
    return MGWR_OK;
}

const char *mgwr_kernel_name(int kernel)
{
    static thread_local std::string name;
    int mode = kernel >> 4, epi = (kernel >> 1) & 7, narrow = kernel & 1;
    if (mode == GM_BF16X3) name = "k_toep_bf16x3<" + std::to_string(epi) + ">";
    else name = std::string(narrow ? "k_toep_narrow<" : "k_toep_wide<") + std::to_string(mode) + ", " +
                std::to_string(epi) + ">";
    return name.c_str();
}

// ---------------------------------------------------------------------------
// Batches: one handle per problem; the solves advance in lockstep so that one
// host synchronisation per cycle serves every problem of the batch.
}  // extern "C"

struct mgwr_batch_ctx {
    std::vector<mgwr_t> hs;
    hipStream_t stream = nullptr;
};

extern "C" {

int mgwr_batch_create(int count, const int *N, const int *M, const double *alpha, const double *T, int dims,
                      const mgwr_options *opts, mgwr_batch_t *out)
{
    if (!out) return fail(MGWR_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (count < 1 || !N || !M || !alpha || !T) return fail(MGWR_EINVAL, "bad batch description");
    mgwr_batch_ctx *b = new mgwr_batch_ctx();
    for (int i = 0; i < count; ++i) {
        mgwr_t h = nullptr;
        int rc = mgwr_create_ex(N[i], M[i], alpha[i], T[i], dims, opts, &h);
        if (rc < 0) {
            std::string msg = "problem " + std::to_string(i) + ": " + g_err;
            for (auto x : b->hs) mgwr_destroy(x);
            delete b;
            g_err = msg;
            return rc;
        }
        b->hs.push_back(h);
    }
    *out = b;
    return MGWR_OK;
}

int mgwr_batch_set_stream(mgwr_batch_t b, void *hip_stream)
{
    if (!b) return fail(MGWR_EINVAL, "NULL batch");
    b->stream = (hipStream_t)hip_stream;
    for (auto h : b->hs) h->stream = b->stream;
    return MGWR_OK;
}

int mgwr_batch_solve(mgwr_batch_t b, const double *const *f, const double *const *g, double *const *u,
                     double tol, mgwr_info *infos)
{
    if (!b || !f || !u) return fail(MGWR_EINVAL, "NULL argument");
    int worst = MGWR_OK;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        mgwr_info inf;
        int rc = mgwr_solve(b->hs[i], f[i], g ? g[i] : nullptr, u[i], tol, &inf);
        if (infos) infos[i] = inf;
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
    }
    return worst;
}

int mgwr_batch_destroy(mgwr_batch_t b)
{
    if (!b) return MGWR_OK;
    for (auto h : b->hs) mgwr_destroy(h);
    delete b;
    return MGWR_OK;
}

}  // extern "C"
