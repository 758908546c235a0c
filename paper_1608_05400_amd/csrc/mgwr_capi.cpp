// Host runtime and C ABI of the MGWR solver (include/mgwr.h).
//
// Method: Gaspar & Rodrigo, "Multigrid waveform relaxation for the
// time-fractional heat equation", arXiv:1608.05400.  The L1 discretisation
// (Section 2) makes the space-time matrix T_M (x) I + A_h with T_M lower
// triangular Toeplitz (Section 5).  Algorithm 1 (Section 3) is run with
//   * smoother: red-black waveform relaxation; one half-sweep solves
//     (T_M + sigma I) x = b for every point of a colour, either
//       - as one causal Toeplitz product of the precomputed first column of
//         (T_M + sigma I)^{-1} (a lower-triangular Toeplitz matrix, Section
//         5.2) with the colour's right-hand sides, or
//       - by the divide-and-conquer blocked forward substitution of Section
//         5.2: base blocks of Mb rows by the inverse of the leading Mb x Mb
//         block, and after each base block the history update of the rows
//         that depend on it as one full Toeplitz-block product;
//   * defect: one causal Toeplitz product with T_M plus the stencil;
//   * full weighting / linear (bilinear) interpolation, coarsening in space
//     only down to one point, where one sweep is the exact line solve.
// mgwr_solve runs either Algorithm 1 on u directly (MGWR_FP64), or an outer
// iterative refinement whose residual is FP64 with the iterate carried as a
// double-double (hi in the caller's u, lo internal) and whose correction
// comes from one cycle on the error equation in FP64, FP32 or split-BF16.
//
// Execution: every stage (a half-sweep, a residual, a transfer, the norms) is
// issued for a list of (problem, level) tasks with one launch per kernel, so
// a batch of independent problems advances in lockstep, stage by stage.  The
// host logic of an outer iteration is a deterministic function of the active
// problems and the caller's pointers; it is recorded once (argument arrays
// uploaded to a device arena), captured into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "mgwr.h"
#include "mgwr_internal.h"

using namespace mgwr;

namespace mgwr {
int product_kernel_kind(int mode, int M, int P, const TileKnobs &kn);
}

namespace {

thread_local std::string g_err;

// A named range on the host timeline (roctx): a tracer such as
// rocprofv3 --marker-trace shows the solve, each outer iteration and the
// autotuner; without a tracer the calls do nothing.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

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

}  // namespace

// Error reporting for the other translation units (mgwr_last_error).
int mgwr::set_error(int code, const char *msg) { return fail(code, "%s", msg); }

namespace {

// A failed runtime call is reported through the return code; the runtime's
// last-error state is cleared, so that a later launch check does not report
// it again (a failed allocation is not a device fault).
#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (void)hipGetLastError();                                                            \
            return fail(e_ == hipErrorOutOfMemory ? MGWR_ENOMEM : MGWR_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
        }                                                                                       \
    } while (0)

#define CHK(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ < 0) return rc_;   \
    } while (0)

// Split-BF16 products are used only where a launch has at least this many
// columns; narrower levels (the coarse grids) run their products in FP32.
constexpr int kBf16MinCols = 128;
// Base block of MGWR_SMOOTH_DC when neither the options nor the tuner set one.
constexpr int kDcDefault = 1024;
// FP64 products take the FFT route from this many time levels on unless the
// autotuner has chosen per level (dense: 2M flops per element on the matrix
// cores; FFT: about 32 bytes per element per pass, 4 passes up to M = 512,
// 6 from M = 1024).
constexpr int kFftMinM = 1024;
// The same for the FP32 history products of the mixed cycles, against the
// split-BF16 matrix-core products (about 5x faster per flop than FP64).
constexpr int kFftMinMLow = 4096;
constexpr int kFftMinCols = 64;
// The FP32 FFT route of a smoother product only where its history part is
// small against the diagonal (c / sigma <= this): an FFT's rounding error is
// spread evenly over all time levels, and on the coarse levels, where the
// history carries the whole line solve, FP32 error of that kind slows the
// refinement (1D workload, alpha = 0.7: cycle factor 0.06 -> 0.09).  Those
// levels take the FFT route in FP64.
constexpr double kFft32MaxHist = 0.1;
// Bytes of each of the two work arrays of the FFT route (columns beyond what
// fits are transformed in chunks).
constexpr size_t kFftBufCap = (size_t)1 << 30;

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

// DFT of a zero-padded real vector, X[k] = sum_t v[t] exp(-2 pi i t k / L),
// by an iterative radix-2 FFT in long double (L a power of two); the
// coefficient spectra of the FFT route.
std::vector<std::complex<long double>> host_dft(const std::vector<double> &v, int L)
{
    using C = std::complex<long double>;
    std::vector<C> a(L, C(0, 0)), w(L / 2);
    for (size_t t = 0; t < v.size() && (int)t < L; ++t) a[t] = C(v[t], 0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < L / 2; ++k) w[k] = C(cosl(2 * pi * k / L), -sinl(2 * pi * k / L));
    for (int i = 1, j = 0; i < L; ++i) {
        int bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= L; len <<= 1)
        for (int i = 0; i < L; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const C x = a[i + k], y = a[i + k + len / 2] * w[k * (L / len)];
                a[i + k] = x + y;
                a[i + k + len / 2] = x - y;
            }
    return a;
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
    int dc_tuned = 0;                       // base block chosen by the tuner (0: inverse column)
    int fft_tuned = -1;                     // products by FFT (1) or dense (0); -1: size rule
    void *spec_inv = nullptr;               // DFT of the zero-padded inverse column (FFT route)
    void *spec32_inv_h = nullptr;           // FP32 DFT of its history part (mixed cycles)
    void *spec32_inv = nullptr;             // FP32 DFT of the whole column (mgwr_toeplitz_apply)
};

// Tile knobs per product arithmetic (FP64, FP32, split-BF16).
struct Tuning {
    TileKnobs kn[3];
    bool tuned = false;
    double ms_default = 0, ms_tuned = 0;
};

// Per-launch timing of the products.
struct Profiler {
    bool on = false;
    struct Pending { hipEvent_t a, b; mgwr_kernel_record rec; };
    std::vector<Pending> pending;
    std::vector<mgwr_kernel_record> records;
    std::vector<hipEvent_t> pool;

    hipEvent_t take()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    int resolve(hipStream_t s)
    {
        if (pending.empty()) return MGWR_OK;
        HIPCHK(hipStreamSynchronize(s));
        for (auto &p : pending) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
            p.rec.ms = ms;
            records.push_back(p.rec);
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
        return MGWR_OK;
    }
    void release()
    {
        for (auto &p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
        pending.clear();
        pool.clear();
    }
};

// A recorded outer-iteration program: its argument arena and its graph.
struct Program {
    char *arena = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Issues the stages of one handle or one batch.
struct Runner {
    hipStream_t stream = nullptr;   // the caller's stream
    hipStream_t capture = nullptr;  // private stream the graphs are captured on
    int count = 1;                  // problems
    bool graphs = true;
    Profiler prof;
    std::map<std::string, Program> progs;
    std::list<std::string> lru;
    char *arena = nullptr;          // argument arena of eager grouped programs
    size_t arena_cap = 0;
    double *norms_dev = nullptr, *norms_host = nullptr;   // [count][2]
};

void drop_program(Program &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.arena) (void)hipFree(p.arena);
    p = Program{};
}

void clear_programs(Runner &R)
{
    if (R.progs.empty()) return;
    (void)hipStreamSynchronize(R.stream);   // teardown: nothing to report to
    for (auto &kv : R.progs) drop_program(kv.second);
    R.progs.clear();
    R.lru.clear();
}

void release_runner(Runner &R)
{
    clear_programs(R);
    if (R.arena) (void)hipFree(R.arena);
    if (R.norms_dev) (void)hipFree(R.norms_dev);
    if (R.norms_host) (void)hipHostFree(R.norms_host);
    if (R.capture) (void)hipStreamDestroy(R.capture);
    R.prof.release();
    R.arena = nullptr; R.norms_dev = nullptr; R.norms_host = nullptr; R.capture = nullptr;
}

int init_runner(Runner &R, int count)
{
    R.count = count;
    HIPCHK(hipMalloc((void **)&R.norms_dev, sizeof(double) * 2 * count));
    HIPCHK(hipHostMalloc((void **)&R.norms_host, sizeof(double) * 2 * count, hipHostMallocDefault));
    return MGWR_OK;
}

// The context every stage issues its launches through.
struct Exec {
    hipStream_t s;
    Staging *st;        // argument arrays of grouped launches (nullptr: lists of one only)
    Profiler *prof;     // per-launch timing (nullptr: off)
    bool record() const { return st && st->record; }
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
    double *xpanel = nullptr;        // D&C: FP64 solution panel [M][maxPc]
    float *xop32 = nullptr;          // D&C: its FP32 copy
    uint16_t *xpk_hi = nullptr, *xpk_lo = nullptr;   // D&C: its split-BF16 copy
    double *partials = nullptr;      // norm partials: 2 partials_nblk doubles
    long partials_nblk = 0;
    void *part = nullptr;            // split-K partials of the Toeplitz products
    size_t part_cap = 0;
    // FFT route of the FP64 products: transform length, twiddles, spectra, work arrays
    int fft_L = 0;
    void *fft_tw = nullptr, *spec_tm = nullptr;
    void *fft_tw32 = nullptr, *spec32_tm_h = nullptr, *spec32_tm = nullptr;
    void *fft_buf0 = nullptr, *fft_buf1 = nullptr;
    size_t fft_buf_cap = 0;
    Tuning tune;
    Runner run;
    void *scratch = nullptr;         // this device's static scratch (mgwr_toeplitz_apply_static)
    int inner_prec = -1;             // precision the inner buffers exist for
    int inner_dc = 0;                // D&C buffers of the inner precision exist
    std::vector<void *> inner_alloc; // buffers owned by the inner hierarchy
    std::vector<void *> alloc;       // everything else
};

struct mgwr_batch_ctx {
    std::vector<mgwr_t> hs;
    Runner run;
};

namespace {

int dmalloc(std::vector<void *> &list, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // reported here; not left for a later launch check
        return fail(e == hipErrorOutOfMemory ? MGWR_ENOMEM : MGWR_EDEVICE,
                    "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    }
    list.push_back(*p);
    return MGWR_OK;
}

void free_list(std::vector<void *> &list)
{
    for (void *p : list) (void)hipFree(p);
    list.clear();
}

int upload_coef(mgwr_ctx *h, ToepCoef &c, const std::vector<double> &v)
{
    c.n = (int)v.size();
    c.nq = (c.n + 15) / 16 + 4 * kQOff;
    CHK(dmalloc(h->alloc, (void **)&c.d64, sizeof(double) * c.n));
    CHK(dmalloc(h->alloc, (void **)&c.d32, sizeof(float) * c.n));
    CHK(dmalloc(h->alloc, (void **)&c.fhi, sizeof(uint16_t) * 512 * (size_t)c.nq));
    CHK(dmalloc(h->alloc, (void **)&c.flo, sizeof(uint16_t) * 512 * (size_t)c.nq));
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

// HBM bytes a product itself must move: its operand read once, in the
// precision it is handed over, and per output element what its epilogue
// reads and writes (the FFT route's work arrays are counted apart).
double product_bytes(const GemmArgs &a)
{
    double in = 8.0;
    if (a.mode == GM_BF16X3) in = 4.0;                       // hi + lo
    else if (a.mode == GM_F32) in = (a.fft_spec && a.fft_b64) ? 8.0 : 4.0;
    double out = 8.0;
    switch (a.epi) {
    case EPI_STORE: case EPI_SCATTER: out = 8.0; break;
    case EPI_RESID: out = 16.0; break;                        // F, R (U is the operand)
    case EPI_RESID_DD: case EPI_RESID_C: case EPI_RESID_R: out = 24.0; break;
    default: out = 16.0; break;                               // read-modify-write, b + x
    }
    // the right-hand sides computed where the first pass reads them: F and
    // the other colour's values (about one per point) instead of a panel
    if (a.ea.rhs) in = 16.0;
    return (double)a.K * a.P * in + (double)a.M * a.P * out;
}

// Kernel id of a product: (kind << 8) | (mode << 4) | epilogue, kind 0 =
// narrow, 1 = wide 128 x 64, 2 = wide 256 x 64, 3 = split-BF16, 4 = FFT
// route (passes), 5 = FFT route on chip.
int kernel_id(const GemmArgs &a)
{
    const int kind = a.fft_spec ? (fft_on_chip(a) ? 5 : 4) : product_kernel_kind(a.mode, a.M, a.P, a.knobs);
    return (kind << 8) | (a.mode << 4) | a.epi;
}

GemmArgs gemm_base(mgwr_ctx *h, int mode)
{
    GemmArgs a;
    a.mode = mode;
    a.part = h->part;
    a.part_cap = h->part_cap;
    a.knobs = h->tune.kn[mode];
    return a;
}

// Products of a stage: one grouped launch per kernel class; with profiling
// on, each class is bracketed by events.
int run_gemms(Exec &ex, const std::vector<GemmArgs> &as, int level)
{
    if (as.empty()) return MGWR_OK;
    if (!ex.prof || !ex.prof->on) {
        HIPCHK(launch_toep_gemm(as, ex.st, ex.s));
        return MGWR_OK;
    }
    // profiling: one launch (set) per kernel class between two events; the
    // record pass of an eager run takes the same classes in the same order,
    // so that the argument arrays land where the launch pass looks for them
    std::map<int, std::vector<GemmArgs>> cls;
    for (const GemmArgs &a : as)
        if (a.M > 0 && a.P > 0) cls[kernel_id(a)].push_back(a);
    for (auto &kv : cls) {
        if (ex.record()) {
            HIPCHK(launch_toep_gemm(kv.second, ex.st, ex.s));
            continue;
        }
        Profiler::Pending p;
        p.a = ex.prof->take();
        p.b = ex.prof->take();
        if (!p.a || !p.b) return fail(MGWR_EDEVICE, "hipEventCreate failed");
        p.rec = mgwr_kernel_record{};
        p.rec.kernel = kv.first; p.rec.level = level;
        for (const GemmArgs &a : kv.second) {
            p.rec.M = std::max(p.rec.M, a.M);
            p.rec.K = std::max(p.rec.K, a.K);
            p.rec.P += a.P;
            p.rec.flops += product_flops(a);
            p.rec.bytes += product_bytes(a);
            if (a.fft_spec) p.rec.pass_bytes += fft_work_bytes(a);
            ++p.rec.products;
        }
        HIPCHK(hipEventRecord(p.a, ex.s));
        HIPCHK(launch_toep_gemm(kv.second, ex.st, ex.s));
        HIPCHK(hipEventRecord(p.b, ex.s));
        ex.prof->pending.push_back(p);
    }
    if (ex.prof->pending.size() >= 4096) CHK(ex.prof->resolve(ex.s));
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
    if (o->smoother != MGWR_SMOOTH_INVERSE && o->smoother != MGWR_SMOOTH_DC && o->smoother != MGWR_SMOOTH_AUTO)
        return fail(MGWR_EINVAL, "bad smoother");
    if (o->dc_block != 0 && (o->dc_block < 128 || o->dc_block % 128 != 0))
        return fail(MGWR_EINVAL, "dc_block must be 0 or a positive multiple of 128 (got %d)", o->dc_block);
    if (!(o->L > 0) || !std::isfinite(o->L)) return fail(MGWR_EINVAL, "L must be positive");
    if (!(o->stall >= 0) || o->stall >= 1.0) return fail(MGWR_EINVAL, "stall must be in [0, 1)");
    if (o->graph != 0 && o->graph != 1) return fail(MGWR_EINVAL, "graph must be 0 or 1");
    if (o->inner_cycles < 1 || o->inner_cycles > 8) return fail(MGWR_EINVAL, "inner_cycles must be in [1, 8]");
    if (o->fft < 0 || o->fft > 2) return fail(MGWR_EINVAL, "fft must be 0, 1 or 2");
    return MGWR_OK;
}

// FFT route of the FP64 products: twiddles, the spectra of T_M's column and
// of every level's inverse column, and two work arrays.
int alloc_fft(mgwr_t h)
{
    if (h->fft_tw || h->opt.fft == 0 || h->M < 32) return MGWR_OK;
    int L = 64;
    while (L < 2 * h->M) L <<= 1;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> tw(2 * (size_t)L);
    for (int k = 0; k < L; ++k) {
        tw[2 * k] = (double)cosl(2 * pi * k / L);
        tw[2 * k + 1] = (double)-sinl(2 * pi * k / L);
    }
    CHK(dmalloc(h->alloc, &h->fft_tw, sizeof(double) * tw.size()));
    HIPCHK(hipMemcpy(h->fft_tw, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice));
    std::vector<float> tw32(tw.begin(), tw.end());
    CHK(dmalloc(h->alloc, &h->fft_tw32, sizeof(float) * tw32.size()));
    HIPCHK(hipMemcpy(h->fft_tw32, tw32.data(), sizeof(float) * tw32.size(), hipMemcpyHostToDevice));
    // columns: T_M's, then every level's inverse; the FP32 spectra are of
    // the history parts (first entry zero)
    const int nl = (int)h->lv.size();
    std::vector<std::vector<double>> cols(nl + 1), specs(nl + 1), specs_h(nl + 1);
    cols[nl] = h->r_host;
    for (int l = 0; l < nl; ++l) {
        cols[l].resize(h->M);
        HIPCHK(hipMemcpy(cols[l].data(), h->lv[l].inv.d64, sizeof(double) * h->M, hipMemcpyDeviceToHost));
    }
    std::vector<std::thread> th;
    for (int l = 0; l <= nl; ++l)
        th.emplace_back([&, l]() {
            auto X = host_dft(cols[l], L);
            std::vector<double> hist = cols[l];
            hist[0] = 0.0;
            auto Xh = host_dft(hist, L);
            specs[l].resize(2 * (size_t)L);
            specs_h[l].resize(2 * (size_t)L);
            for (int k = 0; k < L; ++k) {
                specs[l][2 * k] = (double)X[k].real();
                specs[l][2 * k + 1] = (double)X[k].imag();
                specs_h[l][2 * k] = (double)Xh[k].real();
                specs_h[l][2 * k + 1] = (double)Xh[k].imag();
            }
        });
    for (auto &t : th) t.join();
    for (int l = 0; l <= nl; ++l) {
        void **dst = (l == nl) ? &h->spec_tm : &h->lv[l].spec_inv;
        CHK(dmalloc(h->alloc, dst, sizeof(double) * specs[l].size()));
        HIPCHK(hipMemcpy(*dst, specs[l].data(), sizeof(double) * specs[l].size(), hipMemcpyHostToDevice));
        std::vector<float> f32(specs_h[l].begin(), specs_h[l].end());
        void **dst32 = (l == nl) ? &h->spec32_tm_h : &h->lv[l].spec32_inv_h;
        CHK(dmalloc(h->alloc, dst32, sizeof(float) * f32.size()));
        HIPCHK(hipMemcpy(*dst32, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice));
        std::vector<float> g32(specs[l].begin(), specs[l].end());
        void **dstf = (l == nl) ? &h->spec32_tm : &h->lv[l].spec32_inv;
        CHK(dmalloc(h->alloc, dstf, sizeof(float) * g32.size()));
        HIPCHK(hipMemcpy(*dstf, g32.data(), sizeof(float) * g32.size(), hipMemcpyHostToDevice));
    }
    const size_t need = (size_t)16 * L * ((h->lv.back().P + 1) / 2);
    h->fft_buf_cap = std::min(need, kFftBufCap);
    CHK(dmalloc(h->alloc, &h->fft_buf0, h->fft_buf_cap));
    CHK(dmalloc(h->alloc, &h->fft_buf1, h->fft_buf_cap));
    h->fft_L = L;
    return MGWR_OK;
}

// Whether the products of level lev in arithmetic `mode` take the FFT route.
bool fft_for(const mgwr_ctx *h, int lev, int mode = GM_F64)
{
    if (!h->fft_tw || h->opt.fft == 0) return false;
    if (h->opt.fft == 2) return true;
    // the tuner times the cycle's own products: in the mixed modes those are
    // the FP32 / split-BF16 ones, so the FP64 residual keeps the size rule
    const bool cycle_f64 = h->opt.precision == MGWR_FP64 || h->opt.precision == MGWR_FP64_REFINED;
    if (h->lv[lev].fft_tuned >= 0 && (mode != GM_F64 || cycle_f64)) return h->lv[lev].fft_tuned == 1;
    // a transform is several launches over the whole length: not for the
    // few-column products of the coarse levels
    return h->M >= (mode == GM_F64 ? kFftMinM : kFftMinMLow) && h->lv[lev].P >= kFftMinCols;
}

// FFT route of an FP64 product (spec: FP64 spectrum of the full column).
void set_fft(const mgwr_ctx *h, GemmArgs &a, const void *spec)
{
    a.fft_spec = spec;
    a.fft_tw = h->fft_tw;
    a.fft_L = a.fft_Ltw = h->fft_L;
    a.fft_buf0 = h->fft_buf0;
    a.fft_buf1 = h->fft_buf1;
    a.fft_buf_cap = h->fft_buf_cap;
}

// FFT route in FP32 of a history product of the mixed cycles (spec32: FP32
// spectrum of the history column; b64: B is FP64, else FP32).
void set_fft32(const mgwr_ctx *h, GemmArgs &a, const void *spec32, bool b64)
{
    set_fft(h, a, spec32);
    a.mode = GM_F32;
    a.fft_tw = h->fft_tw32;
    a.fft_b64 = b64;
}

// Base block of the line solve on level lev (0: one product with the inverse
// column).  A block that covers all M rows is the inverse-column solve.
int dc_block_of(const mgwr_ctx *h, int lev)
{
    int b = 0;
    if (h->opt.smoother == MGWR_SMOOTH_DC)
        b = h->opt.dc_block > 0 ? h->opt.dc_block : (h->tune.tuned ? h->lv[lev].dc_tuned : kDcDefault);
    else if (h->opt.smoother == MGWR_SMOOTH_AUTO)
        b = h->tune.tuned ? h->lv[lev].dc_tuned : 0;
    return (b > 0 && b < h->M) ? b : 0;
}

bool uses_dc(const mgwr_ctx *h)
{
    return h->opt.smoother != MGWR_SMOOTH_INVERSE;
}

// Buffers the cycle in precision `prec` needs: the inner hierarchy of the
// refinement (FP64 in every precision; FP32 / split-BF16 appear only as
// product operands) and, when the smoother may use D&C, its panels.
int alloc_inner(mgwr_t h, int prec, bool dc)
{
    if (h->inner_prec == prec && h->inner_dc == (int)dc) return MGWR_OK;
    HIPCHK(hipDeviceSynchronize());
    free_list(h->inner_alloc);
    for (auto &L : h->lv) { L.e = nullptr; L.fe = nullptr; }
    h->rs64 = nullptr; h->panel32 = nullptr; h->op32 = nullptr;
    h->pk_hi = h->pk_lo = nullptr;
    h->xpanel = nullptr; h->xop32 = nullptr; h->xpk_hi = h->xpk_lo = nullptr;
    h->inner_prec = -1;
    const long M = h->M;
    const int nl = (int)h->lv.size();
    const long Pf = h->lv.back().P;
    auto &A = h->inner_alloc;
    if (prec != MGWR_FP64) {
        for (int l = 0; l < nl; ++l) {
            CHK(dmalloc(A, (void **)&h->lv[l].e, sizeof(double) * M * h->lv[l].P));
            if (l < nl - 1) CHK(dmalloc(A, (void **)&h->lv[l].fe, sizeof(double) * M * h->lv[l].P));
        }
        h->lv.back().fe = h->res64;   // the outer residual is the finest right-hand side
        CHK(dmalloc(A, (void **)&h->rs64, sizeof(double) * M * Pf));
    }
    const bool low = (prec == MGWR_MIXED_FP32 || prec == MGWR_MIXED_BF16X3);
    if (low) {
        CHK(dmalloc(A, (void **)&h->panel32, sizeof(float) * M * h->maxPc));
        CHK(dmalloc(A, (void **)&h->op32, sizeof(float) * M * Pf));
    }
    h->pk_ld = (Pf + 127) / 128 * 128;
    const size_t pk_bytes = sizeof(uint16_t) * (size_t)h->Mpad * h->pk_ld;
    if (prec == MGWR_MIXED_BF16X3) {
        CHK(dmalloc(A, (void **)&h->pk_hi, pk_bytes));
        CHK(dmalloc(A, (void **)&h->pk_lo, pk_bytes));
    }
    if (dc) {
        CHK(dmalloc(A, (void **)&h->xpanel, sizeof(double) * M * h->maxPc));
        if (low) CHK(dmalloc(A, (void **)&h->xop32, sizeof(float) * M * h->maxPc));
        if (prec == MGWR_MIXED_BF16X3) {
            CHK(dmalloc(A, (void **)&h->xpk_hi, pk_bytes));
            CHK(dmalloc(A, (void **)&h->xpk_lo, pk_bytes));
        }
    }
    h->inner_prec = prec;
    h->inner_dc = dc;
    return MGWR_OK;
}

// ---------------------------------------------------------------------------
// A cycle over a hierarchy whose per-level iterate/rhs are given (FP64).
struct Hier {
    mgwr_ctx *h = nullptr;
    int prec = MGWR_FP64;         // precision of the products (enum mgwr_precision)
    std::vector<double *> u, f;   // per level
    const double *g = nullptr;    // initial condition on the finest level (natural order)
    double *rscratch = nullptr;   // residual scratch [M][P_fine]
    // storage order of every level (lay_pos): the refinement's inner
    // hierarchy keeps each level split by colour, so that the points of a
    // half-sweep and the neighbours its right-hand sides read are contiguous;
    // the plain FP64 hierarchy, whose finest level is the caller's array,
    // keeps the natural order
    int split = 0;
};
struct Task {
    Hier *H;
    int lev;
    bool zero = false;   // the level's iterate is zero on entry to the cycle
};

int level_mode(const Hier &H, long cols)
{
    if (H.prec == MGWR_FP64 || H.prec == MGWR_FP64_REFINED) return GM_F64;
    if (H.prec == MGWR_MIXED_BF16X3 && cols >= kBf16MinCols) return GM_BF16X3;
    return GM_F32;
}

long packed_ld(long cols)
{
    return (cols + 127) / 128 * 128;
}

// Divide-and-conquer line solves (Section 5.2) of one colour for several
// problems at once.  Rows are cut into nb base blocks of Mb; after base block
// j is solved, the rows of the D&C node split at m = j + 1 (leaves
// [m - lowbit(m), m + lowbit(m)) clipped to nb, as for a recursive halving)
// receive the history of leaves [m - lowbit(m), m): B[bottom] -= T X[top],
// one full Toeplitz block with coefficient offset lowbit(m) Mb.
struct DcItem {
    Task t;
    int colour;
};

int dc_half_sweep(Exec &ex, const std::vector<DcItem> &items)
{
    std::vector<RhsArgs> rhs;
    int nbmax = 0;
    for (const DcItem &d : items) {
        mgwr_ctx *h = d.t.H->h;
        Level &L = h->lv[d.t.lev];
        const bool fine = (d.t.lev == (int)h->lv.size() - 1);
        const int Pc = L.Pc[d.colour];
        rhs.push_back(RhsArgs{0, h->dims, L.n, d.colour, h->M, h->Mpad, d.t.H->f[d.t.lev], d.t.H->u[d.t.lev],
                              h->cd, fine ? d.t.H->g : nullptr, L.ih2, 0.0, h->panel64, nullptr, Pc});
        rhs.back().split = d.t.H->split;
        const int Mb = dc_block_of(h, d.t.lev);
        nbmax = std::max(nbmax, (h->M + Mb - 1) / Mb);
    }
    HIPCHK(launch_rhs(rhs, ex.st, ex.s));
    for (int j = 0; j < nbmax; ++j) {
        std::vector<OperandArgs> prep, xconv;
        std::vector<GemmArgs> leaf, upd;
        int level = -1;
        for (const DcItem &d : items) {
            mgwr_ctx *h = d.t.H->h;
            Level &L = h->lv[d.t.lev];
            level = d.t.lev;
            const int Mb = dc_block_of(h, d.t.lev), nb = (h->M + Mb - 1) / Mb;
            if (j >= nb) continue;
            const int Pc = L.Pc[d.colour];
            const long ldp = packed_ld(Pc);
            const int mode = level_mode(*d.t.H, Pc);
            const int a0 = j * Mb, cnt = std::min(Mb, h->M - a0);
            const int cnt32 = (cnt + 31) / 32 * 32;
            GemmArgs g = gemm_base(h, mode);
            g.M = cnt; g.P = Pc; g.K = cnt; g.off = 0;
            g.ea.out = h->xpanel + (long)a0 * Pc; g.ea.ldo = Pc;
            if (mode == GM_F64) {
                g.coef = &L.inv; g.epi = EPI_STORE; g.B = h->panel64 + (long)a0 * Pc; g.ldb = Pc;
            } else if (mode == GM_F32) {
                prep.push_back(OperandArgs{1, cnt, cnt, Pc, h->panel64 + (long)a0 * Pc, Pc,
                                           h->op32 + (long)a0 * Pc, nullptr, Pc, h->xpanel + (long)a0 * Pc, L.lam0});
                g.coef = &L.inv_h; g.epi = EPI_ADD; g.B = h->op32 + (long)a0 * Pc; g.ldb = Pc;
                if (j + 1 < nb)
                    xconv.push_back(OperandArgs{1, cnt, cnt, Pc, h->xpanel + (long)a0 * Pc, Pc,
                                                h->xop32 + (long)a0 * Pc, nullptr, Pc, nullptr, 0.0});
            } else {
                prep.push_back(OperandArgs{2, cnt, cnt32, Pc, h->panel64 + (long)a0 * Pc, Pc, h->pk_hi + a0 * ldp,
                                           h->pk_lo + a0 * ldp, ldp, h->xpanel + (long)a0 * Pc, L.lam0});
                g.coef = &L.inv_h; g.epi = EPI_ADD;
                g.Bhi = h->pk_hi + a0 * ldp; g.Blo = h->pk_lo + a0 * ldp; g.ldb = ldp;
                if (j + 1 < nb)
                    xconv.push_back(OperandArgs{2, cnt, cnt32, Pc, h->xpanel + (long)a0 * Pc, Pc,
                                                h->xpk_hi + a0 * ldp, h->xpk_lo + a0 * ldp, ldp, nullptr, 0.0});
            }
            leaf.push_back(g);
            if (j + 1 < nb) {
                const int m = j + 1, lb = m & -m, l0 = m - lb, l1 = std::min(m + lb, nb);
                const int r0 = m * Mb, r1 = std::min(l1 * Mb, h->M), k0 = l0 * Mb;
                GemmArgs u = gemm_base(h, mode);
                u.M = r1 - r0; u.P = Pc; u.K = lb * Mb; u.off = lb * Mb; u.coef = &h->tm;
                u.epi = EPI_SUB; u.ea.out = h->panel64 + (long)r0 * Pc; u.ea.ldo = Pc;
                if (mode == GM_F64) { u.B = h->xpanel + (long)k0 * Pc; u.ldb = Pc; }
                else if (mode == GM_F32) { u.B = h->xop32 + (long)k0 * Pc; u.ldb = Pc; }
                else { u.Bhi = h->xpk_hi + k0 * ldp; u.Blo = h->xpk_lo + k0 * ldp; u.ldb = ldp; }
                upd.push_back(u);
            }
        }
        HIPCHK(launch_operand(prep, ex.st, ex.s));
        CHK(run_gemms(ex, leaf, level));
        HIPCHK(launch_operand(xconv, ex.st, ex.s));
        CHK(run_gemms(ex, upd, level));
    }
    std::vector<ScatterArgs> sc;
    for (const DcItem &d : items) {
        mgwr_ctx *h = d.t.H->h;
        Level &L = h->lv[d.t.lev];
        sc.push_back(ScatterArgs{h->dims, L.n, d.colour, h->M, L.Pc[d.colour], h->xpanel, d.t.H->u[d.t.lev],
                                 d.t.H->split});
    }
    HIPCHK(launch_scatter(sc, ex.st, ex.s));
    return MGWR_OK;
}

// One half-sweep (colour `rank` 0 = first, 1 = second) of every task: every
// point of the colour gets the solution of (T_M + sigma I) x = b along its
// time line.  Inverse-column solve: in FP64 the product is the whole solve;
// in FP32 / split-BF16 the right-hand-side kernel writes lambda_0 b (FP64)
// into the colour's points and the product adds the history part.
int half_sweep(Exec &ex, const std::vector<Task> &ts, int rank)
{
    std::vector<RhsArgs> rhs;
    std::vector<GemmArgs> prods;
    std::vector<DcItem> dcs;
    int level = -1;
    for (const Task &t : ts) {
        mgwr_ctx *h = t.H->h;
        Level &L = h->lv[t.lev];
        const int colour = rank == 0 ? h->opt.first_colour : 1 - h->opt.first_colour;
        const int Pc = L.Pc[colour];
        if (Pc == 0) continue;
        level = t.lev;
        if (dc_block_of(h, t.lev) > 0) {
            dcs.push_back(DcItem{t, colour});
            continue;
        }
        const bool fine = (t.lev == (int)h->lv.size() - 1);
        const double *g = fine ? t.H->g : nullptr;
        const int mode = level_mode(*t.H, Pc);
        const int split = t.H->split;
        const long off = split ? lay_cpos(h->dims, L.n, 1, colour, 0) : 0;   // the colour's first point
        GemmArgs a = gemm_base(h, mode);
        a.M = h->M; a.P = Pc; a.K = h->M; a.off = 0;
        a.ea.out = t.H->u[t.lev]; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n; a.ea.colour = colour;
        // On the FFT route, a zero iterate (first half-sweep of a level that
        // starts from zero, no initial-condition term) makes the right-hand
        // sides the colour's points of F: the products read them there and
        // no panel is built; the right-hand-side kernels of the other routes
        // read no neighbours then.
        const bool from_f = t.zero && !g;
        auto push_rhs = [&](RhsArgs r) {
            r.split = split;
            r.zero_nbrs = from_f ? 1 : 0;
            rhs.push_back(r);
        };
        auto rhs_panel = [&]() {
            if (from_f && split) {
                a.B = t.H->f[t.lev] + off; a.ldb = L.P;
            } else if (split && a.mode == GM_F64) {
                // FP64 route: the passes compute the right-hand sides where
                // they read them (F and the other colour's values instead of
                // a panel: 9 % less time per FP64-refinement step on the 1D
                // N = 4095, M = 16384 problems).  Not on the FP32 route, whose
                // last pass needs b again for the diagonal term: computing it
                // there too measured 6 % slower per step (83.0 -> 88.0 ms),
                // with 16 column pairs per block in the first pass
                a.B = t.H->f[t.lev] + off; a.ldb = L.P;
                a.ea.rhs = 1;
                a.ea.F = t.H->f[t.lev] + off; a.ea.U = t.H->u[t.lev]; a.ea.ldu = L.P;
                a.ea.cd = h->cd; a.ea.g = g; a.ea.ih2 = L.ih2;
            } else if (from_f) {
                a.B = t.H->f[t.lev]; a.ldb = L.P; a.b_colour = colour;
            } else {
                push_rhs(RhsArgs{0, h->dims, L.n, colour, h->M, h->Mpad, t.H->f[t.lev], t.H->u[t.lev], h->cd,
                                 g, L.ih2, 0.0, h->panel64, nullptr, Pc});
                a.B = h->panel64; a.ldb = Pc;
            }
        };
        if (mode == GM_F64 && fft_for(h, t.lev)) {
            a.coef = &L.inv; a.epi = EPI_SCATTER;
            set_fft(h, a, L.spec_inv);
            rhs_panel();
        } else if (mode == GM_F64) {
            push_rhs(RhsArgs{0, h->dims, L.n, colour, h->M, h->Mpad, t.H->f[t.lev], t.H->u[t.lev], h->cd, g,
                             L.ih2, 0.0, h->panel64, nullptr, Pc});
            a.coef = &L.inv; a.epi = EPI_SCATTER; a.B = h->panel64; a.ldb = Pc;
        } else if (fft_for(h, t.lev, mode) && h->c > kFft32MaxHist * L.sigma) {
            a.mode = GM_F64; a.coef = &L.inv; a.epi = EPI_SCATTER;
            set_fft(h, a, L.spec_inv);
            rhs_panel();
        } else if (fft_for(h, t.lev, mode)) {
            // FP64 right-hand sides; the FFT's first pass rounds them to FP32
            // and its last pass writes lambda_0 b + history into the colour's
            // contiguous points of U (one store, the diagonal term in FP64)
            a.coef = &L.inv_h; a.epi = EPI_STORE_DIAG; a.ea.diag = L.lam0;
            set_fft32(h, a, L.spec32_inv_h, true);
            rhs_panel();
            a.ea.b = (const double *)a.B; a.ea.ldb_diag = a.ldb;
        } else if (mode == GM_F32) {
            push_rhs(RhsArgs{1, h->dims, L.n, colour, h->M, h->Mpad, t.H->f[t.lev], t.H->u[t.lev], h->cd, g,
                             L.ih2, L.lam0, h->panel32, nullptr, Pc});
            a.coef = &L.inv_h; a.epi = EPI_ADD; a.B = h->panel32; a.ldb = Pc;
        } else {
            const long ldp = packed_ld(Pc);
            push_rhs(RhsArgs{2, h->dims, L.n, colour, h->M, h->Mpad, t.H->f[t.lev], t.H->u[t.lev], h->cd, g,
                             L.ih2, L.lam0, h->pk_hi, h->pk_lo, ldp});
            a.coef = &L.inv_h; a.epi = EPI_ADD; a.Bhi = h->pk_hi; a.Blo = h->pk_lo; a.ldb = ldp;
        }        if (split) {
            // the colour's points are contiguous from `off`: the FP64 route's
            // scatter is a plain store there
            a.ea.out = t.H->u[t.lev] + off;
            if (a.epi == EPI_SCATTER) a.epi = EPI_STORE;
        } else if (a.epi != EPI_SCATTER) {
            // the low-precision epilogues write a colour's contiguous points:
            // only the refinement's inner hierarchy (split) runs them
            return fail(MGWR_EINVAL, "low-precision smoothing on a level in natural order");
        }
        prods.push_back(a);
    }
    HIPCHK(launch_rhs(rhs, ex.st, ex.s));
    CHK(run_gemms(ex, prods, level));
    if (!dcs.empty()) CHK(dc_half_sweep(ex, dcs));
    return MGWR_OK;
}

int sweep(Exec &ex, const std::vector<Task> &ts)
{
    if (ts.empty()) return MGWR_OK;
    CHK(half_sweep(ex, ts, 0));
    // after the first half-sweep no iterate is zero
    std::vector<Task> ts1 = ts;
    for (Task &t : ts1) t.zero = false;
    CHK(half_sweep(ex, ts1, 1));
    return MGWR_OK;
}

// Whether the residual of a task's level takes the FFT route.
bool residual_fft(const Task &t)
{
    const int mode = level_mode(*t.H, t.H->h->lv[t.lev].P);
    return mode == GM_F64 ? fft_for(t.H->h, t.lev) : fft_for(t.H->h, t.lev, mode);
}

// Whether the residual before restriction is computed at one colour only.
// After a red-black sweep the second colour's line solves have made its
// residual zero up to their rounding, so with pre-smoothing the inner cycles
// of the refinement compute only the first colour's residual, on the FFT
// route, which reads those columns directly; the restriction then reads that
// colour alone.  Not in plain FP64 cycles: the FFT route's rounding is
// relative to the largest terms of a time line, so at the early time levels
// the line solves' residual is not small against the local values, and
// Algorithm 1 on the iterate itself has no outer FP64 residual to correct
// for leaving it out (measured: error 5e-10 against 4e-12 on the 1D
// N = 4095, M = 16384 problem).
bool colour_residual(const Task &t)
{
    return t.H->prec != MGWR_FP64 && t.H->h->opt.nu1 >= 1 && residual_fft(t);
}

// A level that starts the cycle from zero and is pre-smoothed by one
// red-black sweep needs no residual product: the first half-sweep solved the
// first colour's line systems with zero neighbours, so after the second
// half-sweep the first colour's residual is ih2 times the neighbour sum of
// the second colour's new values, and the second colour's residual is zero
// (exact in exact arithmetic; its rounding is that of the line solves).  The
// restriction computes it on the fly from the iterate.
bool implicit_residual(const Task &t)
{
    return t.zero && t.H->h->opt.nu1 == 1;
}

// In 1D with colour 0 relaxed first, the colour-0 points are exactly the
// coarse points, so full weighting of a residual that is zero at colour 1
// is 0.25 (2 r) at each of them: the residual kernel writes the coarse
// right-hand side itself.
bool restricted_residual(const Task &t)
{
    return colour_residual(t) && t.H->h->dims == 1 && t.H->h->opt.first_colour == 0;
}

// out = f + c d g - T_M u - A_h u on each task's level: the Toeplitz product
// (all of T_M u in FP64, its history part otherwise) stored into out, then the
// stencil part and the diagonal r_1 u applied by a bandwidth kernel (on the
// FFT route by the product's last pass; at the first colour's points only
// where colour_residual holds).
int level_residual(Exec &ex, const std::vector<Task> &ts)
{
    std::vector<OperandArgs> ops;
    std::vector<GemmArgs> prods;
    std::vector<PostArgs> posts;
    int level = -1;
    for (const Task &t : ts) {
        mgwr_ctx *h = t.H->h;
        Level &L = h->lv[t.lev];
        const bool fine = (t.lev == (int)h->lv.size() - 1);
        level = t.lev;
        const int mode = level_mode(*t.H, L.P);
        double *out = t.H->rscratch;
        const int split = t.H->split;
        GemmArgs a = gemm_base(h, mode);
        a.M = h->M; a.P = (int)L.P; a.K = h->M; a.off = 0; a.epi = EPI_STORE;
        a.ea.out = out; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n;
        a.ea.lay_in = a.ea.lay_out = split;
        if (mode == GM_F64) {
            a.coef = &h->tm; a.B = t.H->u[t.lev]; a.ldb = L.P;
            if (fft_for(h, t.lev)) set_fft(h, a, h->spec_tm);
        } else if (fft_for(h, t.lev, mode)) {
            // the FFT's first pass reads the FP64 iterate itself
            a.coef = &h->tm_h; a.B = t.H->u[t.lev]; a.ldb = L.P;
            set_fft32(h, a, h->spec32_tm_h, true);
        } else if (mode == GM_F32) {
            ops.push_back(OperandArgs{1, h->M, h->M, (int)L.P, t.H->u[t.lev], L.P, h->op32, nullptr, L.P, nullptr, 0.0});
            a.coef = &h->tm_h; a.B = h->op32; a.ldb = L.P;
        } else {
            const long ldp = packed_ld(L.P);
            ops.push_back(OperandArgs{2, h->M, h->Mpad, (int)L.P, t.H->u[t.lev], L.P, h->pk_hi, h->pk_lo, ldp,
                                      nullptr, 0.0});
            a.coef = &h->tm_h; a.Bhi = h->pk_hi; a.Blo = h->pk_lo; a.ldb = ldp;
        }
        const double diag = (a.mode == GM_F64) ? 0.0 : h->c;
        if (a.fft_spec) {
            // FFT route: its last pass applies the stencil part itself
            a.epi = EPI_RESID;
            a.ea.F = t.H->f[t.lev]; a.ea.U = t.H->u[t.lev]; a.ea.lo = nullptr; a.ea.cd = h->cd;
            a.ea.g = fine ? t.H->g : nullptr; a.ea.ih2 = L.ih2; a.ea.diag = diag; a.ea.ldu = L.P;
            if (colour_residual(t)) {
                const int colour = h->opt.first_colour;
                a.epi = EPI_RESID_C;
                a.P = L.Pc[colour];
                if (split) a.B = t.H->u[t.lev] + lay_cpos(h->dims, L.n, 1, colour, 0);   // contiguous
                else a.b_colour = colour;
                a.ea.colour = colour;
                if (restricted_residual(t)) {
                    a.epi = EPI_RESID_R;
                    a.ea.out = t.H->f[t.lev - 1];
                    a.ea.ldo = h->lv[t.lev - 1].P;
                }
            }
            prods.push_back(a);
            continue;
        }
        prods.push_back(a);
        posts.push_back(PostArgs{h->dims, L.n, h->M, t.H->f[t.lev], t.H->u[t.lev], nullptr, h->cd,
                                 fine ? t.H->g : nullptr, L.ih2, diag, out, split, split});
    }
    HIPCHK(launch_operand(ops, ex.st, ex.s));
    CHK(run_gemms(ex, prods, level));
    HIPCHK(launch_post(posts, ex.st, ex.s));
    return MGWR_OK;
}

// One cycle of Algorithm 1 for every task (each on its own level): the tasks
// at their coarsest level do the exact one-point solve while the others
// pre-smooth, then the others recurse together.
// A level that starts a cycle from zero needs no zero fill when every point
// is written before it is read: pre-smoothing comes first, and its first
// half-sweep (no initial-condition term) takes its right-hand sides from F
// alone (the FFT route's products read F's colour points, the right-hand-side
// kernels of the dense routes read no neighbours) and writes the colour's
// points before any read of them; the second half-sweep reads only those.
// (The D&C half-sweep builds its right-hand sides from the iterate.)
bool skip_zero_fill(const Hier &H, int lev)
{
    const mgwr_ctx *h = H.h;
    if (h->opt.nu1 < 1 || dc_block_of(h, lev) > 0) return false;
    if (lev == (int)h->lv.size() - 1 && H.g) return false;
    return h->lv[lev].Pc[h->opt.first_colour] > 0;
}

int cycle(Exec &ex, const std::vector<Task> &ts)
{
    if (ts.empty()) return MGWR_OK;
    std::vector<Task> fine;
    int nu1 = 0, nu2 = 0, gam = 0;
    for (const Task &t : ts) {
        const mgwr_options &o = t.H->h->opt;
        if (t.lev > 0) {
            fine.push_back(t);
            nu1 = std::max(nu1, o.nu1);
            nu2 = std::max(nu2, o.nu2);
            gam = std::max(gam, o.gamma);
        } else {
            nu1 = std::max(nu1, 1);
        }
    }
    for (int i = 0; i < nu1; ++i) {
        std::vector<Task> sel;
        for (const Task &t : ts)
            if ((t.lev > 0 && i < t.H->h->opt.nu1) || (t.lev == 0 && i == 0)) {
                sel.push_back(t);
                if (i > 0) sel.back().zero = false;
            }
        CHK(sweep(ex, sel));
    }
    if (fine.empty()) return MGWR_OK;
    std::vector<Task> explicit_res;
    for (const Task &t : fine)
        if (!implicit_residual(t)) explicit_res.push_back(t);
    CHK(level_residual(ex, explicit_res));
    std::vector<XferArgs> rs, pr;
    std::vector<FillArgs> zs;
    for (const Task &t : fine) {
        mgwr_ctx *h = t.H->h;
        const Level &L = h->lv[t.lev];
        if (implicit_residual(t)) {
            // the residual is ih2 times the neighbour sum of the second colour
            // at the first colour's points (zero at the second's)
            XferArgs x{0, h->dims, L.n, h->M, t.H->u[t.lev], t.H->f[t.lev - 1], 1 - h->opt.first_colour, t.H->split};
            x.implicit = 1;
            x.ih2 = L.ih2;
            rs.push_back(x);
        } else if (!restricted_residual(t)) {
            rs.push_back(XferArgs{0, h->dims, L.n, h->M, t.H->rscratch, t.H->f[t.lev - 1],
                                  colour_residual(t) ? 1 - h->opt.first_colour : -1, t.H->split});
        }
        if (!skip_zero_fill(*t.H, t.lev - 1))
            zs.push_back(FillArgs{h->M, h->lv[t.lev - 1].P, nullptr, nullptr, t.H->u[t.lev - 1], 0});
        XferArgs x{1, h->dims, h->lv[t.lev - 1].n, h->M, t.H->u[t.lev - 1], t.H->u[t.lev], -1, t.H->split};
        // the post-smoothing's first half-sweep recomputes the first colour
        // from the second alone: its correction would be overwritten unread
        if (h->opt.nu2 >= 1) x.skip_colour = h->opt.first_colour;
        pr.push_back(x);
    }
    HIPCHK(launch_xfer(rs, ex.st, ex.s));
    HIPCHK(launch_fill(zs, ex.st, ex.s));
    for (int k = 0; k < gam; ++k) {
        std::vector<Task> down;
        for (const Task &t : fine)
            if (k < t.H->h->opt.gamma) down.push_back(Task{t.H, t.lev - 1, k == 0});   // zero only at the first visit
        CHK(cycle(ex, down));
    }
    HIPCHK(launch_xfer(pr, ex.st, ex.s));
    for (int i = 0; i < nu2; ++i) {
        std::vector<Task> sel;
        for (const Task &t : fine)
            if (i < t.H->h->opt.nu2) {
                sel.push_back(t);
                sel.back().zero = false;
            }
        CHK(sweep(ex, sel));
    }
    return MGWR_OK;
}

Hier plain_hier(mgwr_t h, const double *f, const double *g, double *u)
{
    Hier H;
    H.h = h; H.prec = MGWR_FP64; H.g = g; H.rscratch = h->res64;
    for (auto &L : h->lv) { H.u.push_back(L.u64); H.f.push_back(L.f64); }
    H.u.back() = u; H.f.back() = (double *)f;
    return H;
}

Hier inner_hier(mgwr_t h, int prec)
{
    Hier H;
    H.h = h; H.prec = prec; H.g = nullptr; H.rscratch = h->rs64; H.split = 1;
    for (auto &L : h->lv) { H.u.push_back(L.e); H.f.push_back(L.fe); }
    return H;
}

// The caller's f and u (natural order) into the finest level of an inner
// hierarchy (split storage), and its iterate back into u.
int enter_inner(Exec &ex, Hier &H, const double *f, const double *u)
{
    mgwr_ctx *h = H.h;
    const int top = (int)h->lv.size() - 1;
    HIPCHK(launch_permute({PermuteArgs{h->dims, h->lv[top].n, h->M, 1, f, H.f[top]},
                           PermuteArgs{h->dims, h->lv[top].n, h->M, 1, u, H.u[top]}},
                          nullptr, ex.s));
    return MGWR_OK;
}

int leave_inner(Exec &ex, Hier &H, double *u)
{
    mgwr_ctx *h = H.h;
    const int top = (int)h->lv.size() - 1;
    HIPCHK(launch_permute({PermuteArgs{h->dims, h->lv[top].n, h->M, 0, H.u[top], u}}, nullptr, ex.s));
    return MGWR_OK;
}

// FP64 residual of the finest level into res64 (double-double iterate when
// lo != nullptr) and its norms into norm2 (device, 2 doubles).
// cold: u is the initial iterate g at every time level (lo zero).  Then
// T_M u = c d_m g exactly (the rows of T_M sum to c d_m), so the product is
// replaced by writing c d_m g.
struct FineRes {
    mgwr_ctx *h;
    const double *f, *g, *u, *lo;
    bool cold;
    double *norm2;   // nullptr: no norms
    double *out;     // nullptr: the handle's residual buffer
    int out_split = 0;   // out in the split storage order (the inner hierarchy's right-hand side)
    const double *dd_e = nullptr;   // correction (split order) added to (u, lo) first
};

int fine_residuals(Exec &ex, const std::vector<FineRes> &v)
{
    std::vector<GemmArgs> prods;
    std::vector<FillArgs> fills;
    std::vector<PostArgs> posts;
    std::vector<NormArgs> norms;
    std::vector<DDArgs> upd;
    int level = -1;
    for (const FineRes &r : v) {
        mgwr_ctx *h = r.h;
        Level &L = h->lv.back();
        level = (int)h->lv.size() - 1;
        double *out = r.out ? r.out : h->res64;
        bool fused = false;
        long norm_blocks = 0;   // > 0: the product writes the norm partials
        // the dense route stores the product apart when out is split (the
        // residual kernel reads it in natural order)
        double *prod_at = r.out_split ? h->rs64 : out;
        if (r.cold) {
            fills.push_back(FillArgs{h->M, L.P, h->cd, r.g, prod_at, 1});
        } else {
            GemmArgs a = gemm_base(h, GM_F64);
            a.M = h->M; a.P = (int)L.P; a.K = h->M; a.off = 0; a.coef = &h->tm; a.epi = EPI_STORE;
            a.ea.out = prod_at; a.ea.ldo = L.P; a.ea.dims = h->dims; a.ea.n = L.n;
            a.B = r.u; a.ldb = L.P;
            if (fft_for(h, level)) set_fft(h, a, h->spec_tm);
            // In 1D the FFT route's last pass applies the stencil part itself.
            // In 2D its stencil reads rows n points apart, and the product
            // stored as it is plus the residual kernel take less time
            if (fft_for(h, level) && h->dims == 1) {
                a.epi = r.lo ? EPI_RESID_DD : EPI_RESID;
                a.ea.out = out;
                a.ea.F = r.f; a.ea.U = r.u; a.ea.lo = r.lo; a.ea.cd = h->cd; a.ea.g = r.g;
                a.ea.ih2 = L.ih2; a.ea.diag = 0.0; a.ea.ldu = L.P;
                a.ea.lay_in = 0; a.ea.lay_out = r.out_split;
                fused = true;
                // in one chunk of radix-256 passes the last pass writes the
                // norm partials itself (adding the double-double update to
                // the first pass measured slower than the update kernel:
                // 1.07 ms against 0.33 + 0.55 ms on the 1D N = 4095,
                // M = 16384 problems)
                const long nb = fft_fused_blocks(a);
                if (nb > 0 && r.norm2 && nb <= h->partials_nblk) {
                    a.ea.norm_part = h->partials;
                    norm_blocks = nb;
                }
            }
            prods.push_back(a);
        }
        if (r.dd_e)
            upd.push_back(DDArgs{(long)h->M * L.P, r.dd_e, const_cast<double *>(r.u), const_cast<double *>(r.lo),
                                 h->dims, L.n, 1});
        if (!fused) {
            posts.push_back(PostArgs{h->dims, L.n, h->M, r.f, r.u, r.lo, h->cd, r.g, L.ih2, 0.0, out, 0, r.out_split,
                                     prod_at});
        }
        if (r.norm2) {
            const long n = (long)h->M * L.P;
            if (norm_blocks > 0) norms.push_back(NormArgs{n, out, h->partials, (int)norm_blocks, r.norm2, 1});
            else norms.push_back(NormArgs{n, out, h->partials, norm_partial_blocks(n), r.norm2});
        }
    }
    HIPCHK(launch_fill(fills, ex.st, ex.s));
    HIPCHK(launch_dd_update(upd, ex.st, ex.s));
    CHK(run_gemms(ex, prods, level));
    HIPCHK(launch_post(posts, ex.st, ex.s));
    HIPCHK(launch_norms(norms, ex.st, ex.s));
    return MGWR_OK;
}

// ---------------------------------------------------------------------------
// Programs: run `body` on the runner's stream.  With graphs on (and no
// profiling), the body is recorded once per key: argument arrays into an
// arena of its own, launches captured on a private stream into a graph that
// is replayed on the caller's stream.  Otherwise it runs eagerly (two passes
// when a list has more than one entry).
using Body = std::function<int(Exec &)>;

int run_eager(Runner &R, const Body &body)
{
    if (R.count == 1) {
        Exec ex{R.stream, nullptr, &R.prof};
        return body(ex);
    }
    Staging st;
    st.record = true;
    Exec rec{R.stream, &st, &R.prof};   // (the profiler only decides the order of the records)
    CHK(body(rec));
    if (!st.host.empty()) {
        // earlier launches on the stream may still read the arena
        HIPCHK(hipStreamSynchronize(R.stream));
        if (st.host.size() > R.arena_cap) {
            if (R.arena) (void)hipFree(R.arena);
            R.arena = nullptr;
            R.arena_cap = 0;
            HIPCHK(hipMalloc((void **)&R.arena, st.host.size()));
            R.arena_cap = st.host.size();
        }
        HIPCHK(hipMemcpy(R.arena, st.host.data(), st.host.size(), hipMemcpyHostToDevice));
    }
    st.record = false;
    st.dev = R.arena;
    st.cursor = 0;
    Exec ex{R.stream, &st, &R.prof};
    return body(ex);
}

int run_program(Runner &R, const std::string &key, const Body &body)
{
    if (!R.graphs || R.prof.on) return run_eager(R, body);
    auto it = R.progs.find(key);
    if (it == R.progs.end()) {
        if (R.progs.size() >= 8) {   // keep the 8 most recent
            HIPCHK(hipStreamSynchronize(R.stream));
            drop_program(R.progs[R.lru.front()]);
            R.progs.erase(R.lru.front());
            R.lru.pop_front();
        }
        if (!R.capture) HIPCHK(hipStreamCreateWithFlags(&R.capture, hipStreamNonBlocking));
        Program p;
        Staging st;
        if (R.count > 1) {
            st.record = true;
            Exec rec{R.capture, &st, nullptr};
            CHK(body(rec));
            if (!st.host.empty()) {
                HIPCHK(hipMalloc((void **)&p.arena, st.host.size()));
                hipError_t e = hipMemcpy(p.arena, st.host.data(), st.host.size(), hipMemcpyHostToDevice);
                if (e != hipSuccess) {
                    drop_program(p);
                    HIPCHK(e);
                }
            }
            st.record = false;
            st.dev = p.arena;
            st.cursor = 0;
        }
        Exec ex{R.capture, R.count > 1 ? &st : nullptr, nullptr};
        HIPCHK(hipStreamBeginCapture(R.capture, hipStreamCaptureModeThreadLocal));
        int rc = body(ex);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(R.capture, &graph);
        if (rc < 0 || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            drop_program(p);
            if (rc < 0) return rc;
            HIPCHK(e);
        }
        p.graph = graph;
        e = hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_program(p);
            HIPCHK(e);
        }
        it = R.progs.emplace(key, p).first;
        R.lru.push_back(key);
    } else {
        R.lru.remove(key);
        R.lru.push_back(key);
    }
    HIPCHK(hipGraphLaunch(it->second.exec, R.stream));
    return MGWR_OK;
}

std::string prog_key(const char *kind, const std::vector<int> &active, const std::vector<const void *> &ptrs)
{
    std::string k(kind);
    char buf[32];
    for (int a : active) { snprintf(buf, sizeof buf, ",%d", a); k += buf; }
    k += "|";
    for (const void *p : ptrs) { snprintf(buf, sizeof buf, "%p,", p); k += buf; }
    return k;
}

int read_norms(Runner &R)
{
    HIPCHK(hipMemcpyAsync(R.norms_host, R.norms_dev, sizeof(double) * 2 * R.count, hipMemcpyDeviceToHost,
                          R.stream));
    HIPCHK(hipStreamSynchronize(R.stream));
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

// ---------------------------------------------------------------------------
// The solve of a group of problems (one handle, or a batch) in lockstep: one
// outer iteration (a cycle on u, or a refinement step, and the new residual)
// for every problem that has not stopped, then one read of all norms.
struct SolveState {
    int it = 0, status = MGWR_NOT_CONVERGED, slow = 0;
    double r0 = 0, prev = 0, rn = 0;
    bool done = false;
    mgwr_info inf;
};

void update_state(SolveState &S, const mgwr_options &o, const double nrm[2], double tol)
{
    S.rn = nrm[o.norm];
    if (!std::isfinite(nrm[1]) || !std::isfinite(S.rn)) {
        S.status = MGWR_ENONFINITE;
        S.done = true;
        return;
    }
    if (S.it < 128) S.inf.hist[S.it] = S.rn;
    if (S.it == 0) S.r0 = S.rn;
    if (S.rn <= tol * S.r0) { S.status = MGWR_OK; S.done = true; return; }
    if (S.it > 0 && S.rn > 1e6 * S.r0) { S.status = MGWR_EDIVERGED; S.done = true; return; }
    // Stagnation: a cycle that does not reduce the residual by the factor
    // `stall`.  Near the rounding floor (below 1e-6 r0) one such cycle ends
    // the solve; above it three in a row do (a refinement step may raise the
    // residual once while it removes the smooth error).
    if (S.it > 0 && o.stall > 0 && S.rn > o.stall * S.prev) {
        ++S.slow;
        if (S.rn < 1e-6 * S.r0 || S.slow >= 3) { S.status = MGWR_STAGNATED; S.done = true; return; }
    } else {
        S.slow = 0;
    }
    if (S.it >= o.maxit) { S.status = MGWR_NOT_CONVERGED; S.done = true; return; }
    S.prev = S.rn;
}

int solve_group(Runner &R, const std::vector<mgwr_ctx *> &hs, const double *const *f, const double *const *g,
                double *const *u, double tol, mgwr_info *infos)
{
    TraceRange tr("mgwr solve");
    const int n = (int)hs.size();
    for (mgwr_ctx *h : hs) CHK(alloc_inner(h, h->opt.precision, uses_dc(h)));
    std::vector<Hier> Hp(n), Hi(n);
    std::vector<SolveState> S(n);
    std::vector<const void *> ptrs;
    for (int i = 0; i < n; ++i) {
        mgwr_ctx *h = hs[i];
        Hp[i] = plain_hier(h, f[i], g ? g[i] : nullptr, u[i]);
        if (h->opt.precision != MGWR_FP64) Hi[i] = inner_hier(h, h->opt.precision);
        memset(&S[i].inf, 0, sizeof(mgwr_info));
        ptrs.push_back(f[i]);
        ptrs.push_back(g ? g[i] : nullptr);
        ptrs.push_back(u[i]);
    }
    auto refine = [&](int i) { return hs[i]->opt.precision != MGWR_FP64; };
    auto fine_res = [&](int i, bool cold) {
        mgwr_ctx *h = hs[i];
        return FineRes{h, f[i], g ? g[i] : nullptr, u[i], refine(i) ? h->ulo : nullptr, cold, R.norms_dev + 2 * i,
                       nullptr, refine(i) ? 1 : 0};
    };
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;

    // initial iterate u^0 = g at every time level (Section 3), lo = 0, and
    // the initial residual
    Body init = [&](Exec &ex) -> int {
        std::vector<FillArgs> fills;
        std::vector<FineRes> res;
        for (int i = 0; i < n; ++i) {
            mgwr_ctx *h = hs[i];
            const long P = h->lv.back().P;
            if (!h->opt.warm_start) fills.push_back(FillArgs{h->M, P, nullptr, g ? g[i] : nullptr, u[i], 0});
            if (refine(i)) fills.push_back(FillArgs{h->M, P, nullptr, nullptr, h->ulo, 0});
            res.push_back(fine_res(i, !h->opt.warm_start));
        }
        HIPCHK(launch_fill(fills, ex.st, ex.s));
        return fine_residuals(ex, res);
    };
    CHK(run_program(R, prog_key("init", all, ptrs), init));
    CHK(read_norms(R));
    for (int i = 0; i < n; ++i) update_state(S[i], hs[i]->opt, R.norms_host + 2 * i, tol);

    for (;;) {
        std::vector<int> act;
        for (int i = 0; i < n; ++i)
            if (!S[i].done) act.push_back(i);
        if (act.empty()) break;
        Body step = [&](Exec &ex) -> int {
            std::vector<Task> plain, inner;
            std::vector<FillArgs> zero;
            std::vector<FineRes> res;
            for (int i : act) {
                mgwr_ctx *h = hs[i];
                const int top = (int)h->lv.size() - 1;
                res.push_back(fine_res(i, false));
                if (!refine(i)) {
                    plain.push_back(Task{&Hp[i], top});
                } else {
                    Level &L = h->lv.back();
                    inner.push_back(Task{&Hi[i], top, true});
                    if (!skip_zero_fill(Hi[i], top)) zero.push_back(FillArgs{h->M, L.P, nullptr, nullptr, L.e, 0});
                    res.back().dd_e = L.e;   // u += e (double-double) ahead of the residual
                }
            }
            CHK(cycle(ex, plain));
            HIPCHK(launch_fill(zero, ex.st, ex.s));
            // inner_cycles cycles of the error equation, the first from zero
            int kmax = 0;
            for (const Task &t : inner) kmax = std::max(kmax, t.H->h->opt.inner_cycles);
            for (int k = 0; k < kmax; ++k) {
                std::vector<Task> sel;
                for (const Task &t : inner)
                    if (k < t.H->h->opt.inner_cycles) {
                        sel.push_back(t);
                        sel.back().zero = (k == 0);
                    }
                CHK(cycle(ex, sel));
            }
            return fine_residuals(ex, res);
        };
        {
            TraceRange tr("mgwr outer iteration");
            CHK(run_program(R, prog_key("iter", act, ptrs), step));
        }
        CHK(read_norms(R));
        for (int i : act) {
            ++S[i].it;
            update_state(S[i], hs[i]->opt, R.norms_host + 2 * i, tol);
        }
    }
    HIPCHK(hipStreamSynchronize(R.stream));
    int worst = MGWR_OK;
    for (int i = 0; i < n; ++i) {
        SolveState &s = S[i];
        s.inf.iters = s.it;
        s.inf.status = s.status;
        s.inf.r0 = s.r0;
        s.inf.rk = s.rn;
        s.inf.relres = s.r0 > 0 ? s.rn / s.r0 : 0.0;
        s.inf.mean_factor = (s.it > 0 && s.r0 > 0) ? std::pow(s.rn / s.r0, 1.0 / s.it) : 0.0;
        if (infos) infos[i] = s.inf;
        if (s.status == MGWR_ENONFINITE)
            fail(MGWR_ENONFINITE, "problem %d: non-finite residual after %d cycles", i, s.it);
        else if (s.status == MGWR_EDIVERGED)
            fail(MGWR_EDIVERGED, "problem %d: residual grew from %g to %g", i, s.r0, s.rn);
        if (s.status < 0) worst = std::min(worst, s.status);
        else if (worst >= 0) worst = std::max(worst, s.status);
    }
    return worst;
}

// ---------------------------------------------------------------------------
// Autotuner: times one cycle of the error equation (internal buffers only;
// the caller's arrays are not touched) under candidate tile knobs and D&C
// base blocks, and keeps the fastest.  Results are shared by every handle of
// the same shape and options (process-wide cache).
struct TuneResult {
    TileKnobs kn[3];
    std::vector<int> dc, fft;   // per level
    double ms_default, ms_tuned;
};
std::mutex g_tune_mu;
std::map<std::string, TuneResult> g_tune_cache;

std::string tune_key(const mgwr_ctx *h)
{
    char buf[256];
    snprintf(buf, sizeof buf, "d%d N%d M%d p%d s%d b%d f%d", h->dims, h->N, h->M, h->opt.precision,
             h->opt.smoother, h->opt.dc_block, h->opt.fft);
    return buf;
}

int time_cycle(Runner &R, const std::vector<mgwr_ctx *> &hs, int prec, int reps, double &ms)
{
    std::vector<Hier> H(hs.size());
    for (size_t i = 0; i < hs.size(); ++i) H[i] = inner_hier(hs[i], prec);
    Body body = [&](Exec &ex) -> int {
        std::vector<Task> ts;
        std::vector<FillArgs> zero;
        for (size_t i = 0; i < hs.size(); ++i) {
            Level &L = hs[i]->lv.back();
            ts.push_back(Task{&H[i], (int)hs[i]->lv.size() - 1, true});
            if (!skip_zero_fill(H[i], (int)hs[i]->lv.size() - 1))
                zero.push_back(FillArgs{hs[i]->M, L.P, nullptr, nullptr, L.e, 0});
        }
        HIPCHK(launch_fill(zero, ex.st, ex.s));
        return cycle(ex, ts);
    };
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    ms = 1e30;
    int rc = MGWR_OK;
    const bool prof = R.prof.on;
    R.prof.on = false;
    for (int r = 0; r < reps && rc == MGWR_OK; ++r) {
        hipError_t e = hipEventRecord(a, R.stream);
        if (e == hipSuccess) rc = run_eager(R, body);
        if (e == hipSuccess && rc == MGWR_OK) e = hipEventRecord(b, R.stream);
        if (e == hipSuccess && rc == MGWR_OK) e = hipEventSynchronize(b);
        float t = 0;
        if (e == hipSuccess && rc == MGWR_OK) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess && rc == MGWR_OK)
            rc = fail(MGWR_EDEVICE, "autotuner timing: %s", hipGetErrorString(e));
        if (rc == MGWR_OK) ms = std::min(ms, (double)t);
    }
    R.prof.on = prof;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

// Tuning cache file named by MGWR_TUNE_CACHE (optional): one line per key,
//   key TAB v0 s0 v1 s1 v2 s2 levels dc[levels] fft[levels] ms_default ms_tuned
// (tile variant and split target per product mode); a later line for the
// same key wins.  Unreadable or malformed lines are skipped.
bool tune_file_load(const std::string &key, size_t levels, TuneResult &out)
{
    const char *path = getenv("MGWR_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *fp = fopen(path, "r");
    if (!fp) return false;
    std::vector<char> line(1 << 16);
    bool found = false;
    while (fgets(line.data(), (int)line.size(), fp)) {
        const char *tab = strchr(line.data(), '\t');
        if (!tab || std::string(line.data(), tab - line.data()) != key) continue;
        TuneResult t;
        int v[6], nl = 0, used = 0;
        const char *p = tab + 1;
        if (sscanf(p, "%d %d %d %d %d %d %d%n", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &nl, &used) != 7) continue;
        if (nl != (int)levels) continue;
        p += used;
        bool ok = true;
        for (int m = 0; m < 3; ++m) {
            t.kn[m].variant = v[2 * m];
            t.kn[m].split_target = v[2 * m + 1];
            ok = ok && v[2 * m] >= -1 && v[2 * m] <= 1 && v[2 * m + 1] >= 0;
        }
        t.dc.resize(nl);
        t.fft.resize(nl);
        for (int l = 0; l < nl && ok; ++l) {
            ok = sscanf(p, "%d%n", &t.dc[l], &used) == 1 && t.dc[l] >= 0 && t.dc[l] % 128 == 0;
            p += used;
        }
        for (int l = 0; l < nl && ok; ++l) {
            ok = sscanf(p, "%d%n", &t.fft[l], &used) == 1 && t.fft[l] >= -1 && t.fft[l] <= 1;
            p += used;
        }
        ok = ok && sscanf(p, "%lf %lf", &t.ms_default, &t.ms_tuned) == 2;
        if (ok) {
            out = t;
            found = true;
        }
    }
    fclose(fp);
    return found;
}

void tune_file_store(const std::string &key, const TuneResult &t)
{
    const char *path = getenv("MGWR_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "%s\t", key.c_str());
    for (int m = 0; m < 3; ++m) fprintf(fp, "%d %d ", t.kn[m].variant, t.kn[m].split_target);
    fprintf(fp, "%zu", t.dc.size());
    for (int d : t.dc) fprintf(fp, " %d", d);
    for (int x : t.fft) fprintf(fp, " %d", x);
    fprintf(fp, " %.17g %.17g\n", t.ms_default, t.ms_tuned);
    fclose(fp);
}

int autotune_group(Runner &R, const std::vector<mgwr_ctx *> &hs)
{
    TraceRange range("mgwr autotune");
    mgwr_ctx *h0 = hs[0];
    const std::string key = tune_key(h0);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && hs.size() == 1) {
            for (int m = 0; m < 3; ++m) h0->tune.kn[m] = it->second.kn[m];
            for (size_t l = 0; l < h0->lv.size(); ++l) {
                h0->lv[l].dc_tuned = it->second.dc[l];
                h0->lv[l].fft_tuned = it->second.fft[l];
            }
            h0->tune.ms_default = it->second.ms_default;
            h0->tune.ms_tuned = it->second.ms_tuned;
            h0->tune.tuned = true;
            clear_programs(R);
            return MGWR_OK;
        }
        TuneResult ft;   // a tuning saved by an earlier process
        if (hs.size() == 1 && tune_file_load(key, h0->lv.size(), ft)) {
            g_tune_cache[key] = ft;
            for (int m = 0; m < 3; ++m) h0->tune.kn[m] = ft.kn[m];
            for (size_t l = 0; l < h0->lv.size(); ++l) {
                h0->lv[l].dc_tuned = ft.dc[l];
                h0->lv[l].fft_tuned = ft.fft[l];
            }
            h0->tune.ms_default = ft.ms_default;
            h0->tune.ms_tuned = ft.ms_tuned;
            h0->tune.tuned = true;
            clear_programs(R);
            return MGWR_OK;
        }
    }
    const int prec = h0->opt.precision;
    const int tprec = (prec == MGWR_FP64) ? MGWR_FP64_REFINED : prec;
    for (mgwr_ctx *h : hs) {
        CHK(alloc_inner(h, tprec, uses_dc(h)));
        // start from the choice an untuned handle makes
        for (auto &L : h->lv) {
            L.dc_tuned = (h->opt.smoother == MGWR_SMOOTH_DC) ? kDcDefault : 0;
            L.fft_tuned = -1;
        }
        for (int m = 0; m < 3; ++m) h->tune.kn[m] = TileKnobs{};
        // the finest right-hand side of the error equation: zeros
        std::vector<FillArgs> z{FillArgs{h->M, h->lv.back().P, nullptr, nullptr, h->res64, 0}};
        HIPCHK(launch_fill(z, nullptr, R.stream));
        h->tune.tuned = true;   // dc_block_of reads the tuned blocks from here on
    }
    auto set_kn = [&](int mode, const TileKnobs &k) { for (mgwr_ctx *h : hs) h->tune.kn[mode] = k; };
    // the untuned choices, to fall back on
    struct Snap { TileKnobs kn[3]; std::vector<int> dc, fft; };
    auto snap = [&]() {
        std::vector<Snap> v;
        for (mgwr_ctx *h : hs) {
            Snap x;
            for (int m = 0; m < 3; ++m) x.kn[m] = h->tune.kn[m];
            for (auto &L : h->lv) { x.dc.push_back(L.dc_tuned); x.fft.push_back(L.fft_tuned); }
            v.push_back(x);
        }
        return v;
    };
    auto restore = [&](const std::vector<Snap> &v) {
        for (size_t i = 0; i < hs.size(); ++i) {
            for (int m = 0; m < 3; ++m) hs[i]->tune.kn[m] = v[i].kn[m];
            for (size_t l = 0; l < hs[i]->lv.size(); ++l) {
                hs[i]->lv[l].dc_tuned = v[i].dc[l];
                hs[i]->lv[l].fft_tuned = v[i].fft[l];
            }
        }
    };
    const std::vector<Snap> untuned = snap();
    double best = 0;
    CHK(time_cycle(R, hs, tprec, 2, best));   // also warms up
    CHK(time_cycle(R, hs, tprec, 2, best));
    double ms_default = best;
    std::vector<int> modes;
    if (tprec == MGWR_FP64_REFINED) modes = {GM_F64};
    else if (tprec == MGWR_MIXED_FP32) modes = {GM_F32};
    else modes = {GM_BF16X3, GM_F32};
    for (int mode : modes) {
        if (mode != GM_BF16X3) {
            TileKnobs k = h0->tune.kn[mode];
            for (int v : {0, 1}) {
                TileKnobs c = k;
                c.variant = v;
                set_kn(mode, c);
                double t;
                CHK(time_cycle(R, hs, tprec, 2, t));
                if (t < best * 0.995) { best = t; k = c; }
            }
            set_kn(mode, k);
        }
        TileKnobs k = h0->tune.kn[mode];
        const int base = (mode == GM_BF16X3) ? 1024 : 2048;
        for (int tgt : {base / 4, base / 2, base * 2, base * 4}) {
            TileKnobs c = k;
            c.split_target = tgt;
            set_kn(mode, c);
            double t;
            CHK(time_cycle(R, hs, tprec, 2, t));
            if (t < best * 0.995) { best = t; k = c; }
        }
        set_kn(mode, k);
    }
    int depth = 0;
    for (mgwr_ctx *h : hs) depth = std::max(depth, (int)h->lv.size());
    // FFT or dense route of the products, level by level from the finest
    if (h0->opt.fft == 1 && h0->fft_tw) {
        for (int d = 0; d < depth; ++d) {
            auto set_fft_choice = [&](int c) {
                for (mgwr_ctx *h : hs) {
                    int l = (int)h->lv.size() - 1 - d;
                    if (l >= 0) h->lv[l].fft_tuned = c;
                }
            };
            // the default of the deepest-reaching problem decides where to start
            mgwr_ctx *hp = h0;
            for (mgwr_ctx *h : hs)
                if (h->lv.size() > hp->lv.size()) hp = h;
            const int l0 = (int)hp->lv.size() - 1 - d;
            Hier probe = inner_hier(hp, tprec);
            set_fft_choice(-1);
            const int def = fft_for(hp, l0, level_mode(probe, hp->lv[l0].P)) ? 1 : 0;
            set_fft_choice(def);
            CHK(time_cycle(R, hs, tprec, 2, best));
            set_fft_choice(1 - def);
            double t;
            CHK(time_cycle(R, hs, tprec, 2, t));
            if (t < best * 0.995) best = t;
            else set_fft_choice(def);
        }
    }
    // D&C base blocks, level by level from the finest (the same choice for
    // every problem at the same depth)
    if (h0->opt.smoother != MGWR_SMOOTH_INVERSE && h0->opt.dc_block == 0) {
        std::vector<int> cands;
        if (h0->opt.smoother == MGWR_SMOOTH_AUTO) cands.push_back(0);
        for (int b : {4096, 2048, 1024, 512, 256}) cands.push_back(b);
        for (int d = 0; d < depth; ++d) {
            auto set_dc = [&](int b) {
                for (mgwr_ctx *h : hs) {
                    int l = (int)h->lv.size() - 1 - d;
                    if (l >= 0) h->lv[l].dc_tuned = b;
                }
            };
            int bestb = (h0->opt.smoother == MGWR_SMOOTH_AUTO) ? 0 : kDcDefault;
            set_dc(bestb);
            CHK(time_cycle(R, hs, tprec, 2, best));
            for (int b : cands) {
                if (b == bestb) continue;
                if (b != 0 && b >= h0->M) continue;
                set_dc(b);
                double t;
                CHK(time_cycle(R, hs, tprec, 2, t));
                if (t < best * 0.995) { best = t; bestb = b; }
            }
            set_dc(bestb);
        }
    }
    // the choices against the untuned ones, head to head (stage timings are
    // noisy for short cycles); keep the faster
    {
        const std::vector<Snap> tuned = snap();
        double t_tuned = 0, t_default = 0;
        CHK(time_cycle(R, hs, tprec, 3, t_tuned));
        restore(untuned);
        CHK(time_cycle(R, hs, tprec, 3, t_default));
        ms_default = t_default;
        if (t_tuned < t_default) {
            restore(tuned);
            best = t_tuned;
        } else {
            best = t_default;
        }
    }
    for (mgwr_ctx *h : hs) {
        h->tune.ms_default = ms_default;
        h->tune.ms_tuned = best;
        CHK(alloc_inner(h, prec, uses_dc(h)));
    }
    clear_programs(R);
    if (hs.size() == 1) {
        TuneResult tr;
        for (int m = 0; m < 3; ++m) tr.kn[m] = h0->tune.kn[m];
        for (auto &L : h0->lv) {
            tr.dc.push_back(L.dc_tuned);
            tr.fft.push_back(L.fft_tuned);
        }
        tr.ms_default = ms_default;
        tr.ms_tuned = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = tr;
        tune_file_store(key, tr);
    }
    return MGWR_OK;
}

void tuning_out(const mgwr_ctx *h, mgwr_tuning *t)
{
    memset(t, 0, sizeof *t);
    t->tuned = h->tune.tuned ? 1 : 0;
    t->variant[0] = h->tune.kn[GM_F64].variant;
    t->variant[1] = h->tune.kn[GM_F32].variant;
    for (int m = 0; m < 3; ++m) t->split_target[m] = h->tune.kn[m].split_target;
    t->levels = (int)h->lv.size();
    Hier probe;
    probe.prec = h->opt.precision;
    for (int l = 0; l < t->levels && l < 32; ++l) {
        t->dc_block[l] = dc_block_of(h, l);
        t->fft[l] = fft_for(h, l, level_mode(probe, h->lv[l].P)) ? 1 : 0;
    }
    t->ms_default = h->tune.ms_default;
    t->ms_tuned = h->tune.ms_tuned;
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
    o->smoother = MGWR_SMOOTH_INVERSE; o->dc_block = 0; o->L = 1.0; o->stall = 0.5; o->graph = 1;
    o->fft = 1;
    o->inner_cycles = 1;
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
    // teardown: errors here have no caller to go to
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    (void)hipDeviceSynchronize();
    release_runner(h->run);
    free_list(h->inner_alloc);
    free_list(h->alloc);
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
    h->run.graphs = o.graph != 0;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(MGWR_EDEVICE, "no HIP device available");
    }
    int rc = [&]() -> int {
        CHK(static_scratch(h->device, &h->scratch));
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
        CHK(dmalloc(h->alloc, (void **)&h->cd, sizeof(double) * M));
        HIPCHK(hipMemcpy(h->cd, cdv.data(), sizeof(double) * M, hipMemcpyHostToDevice));
        const long Pf = h->lv.back().P;
        for (size_t l = 0; l + 1 < h->lv.size(); ++l) {
            CHK(dmalloc(h->alloc, (void **)&h->lv[l].u64, sizeof(double) * M * h->lv[l].P));
            CHK(dmalloc(h->alloc, (void **)&h->lv[l].f64, sizeof(double) * M * h->lv[l].P));
        }
        CHK(dmalloc(h->alloc, (void **)&h->res64, sizeof(double) * M * Pf));
        CHK(dmalloc(h->alloc, (void **)&h->panel64, sizeof(double) * M * h->maxPc));
        CHK(dmalloc(h->alloc, (void **)&h->ulo, sizeof(double) * M * Pf));
        // norm partials: the blocks of the reduction kernel, or those of the
        // last pass of the finest FP64 residual product by FFT (which writes them)
        h->partials_nblk = 2048;
        {
            long L = 64;
            while (L < 2L * M) L <<= 1;
            const long Q = (Pf + 1) / 2;
            if (L >= 512) h->partials_nblk = std::max(h->partials_nblk, (Q + 15) / 16 * (L / 256));
        }
        CHK(dmalloc(h->alloc, (void **)&h->partials, sizeof(double) * 2 * h->partials_nblk));
        // split-K scratch: the largest any lone product of this hierarchy
        // needs under any tile knobs the tuner tries
        size_t part = 0;
        for (const Level &L : h->lv)
            for (int mode = GM_F64; mode <= GM_BF16X3; ++mode) {
                long cols[3] = {L.Pc[0], L.Pc[1], L.P};
                for (long P : cols)
                    for (int tgt : {0, 8192})
                        for (int v : {0, 1}) {
                            TileKnobs kn;
                            kn.variant = v;
                            kn.split_target = tgt;
                            if (P > 0) part = std::max(part, splitk_bytes(mode, M, (int)P, M, 0, M, kn));
                        }
            }
        if (part > 0) {
            CHK(dmalloc(h->alloc, &h->part, part));
            h->part_cap = part;
        }
        CHK(init_runner(h->run, 1));
        CHK(alloc_fft(h));
        CHK(alloc_inner(h, o.precision, uses_dc(h)));
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
    clear_programs(h->run);
    mgwr_options old = h->opt;
    h->opt = *opts;
    int rc = alloc_inner(h, opts->precision, uses_dc(h));
    if (rc < 0) {
        h->opt = old;
        return rc;
    }
    h->run.graphs = opts->graph != 0;
    rc = alloc_fft(h);
    if (rc < 0) {
        h->opt = old;
        return rc;
    }
    if (old.precision != opts->precision || old.smoother != opts->smoother || old.dc_block != opts->dc_block ||
        old.fft != opts->fft) {
        h->tune = Tuning{};
        for (auto &L : h->lv) { L.dc_tuned = 0; L.fft_tuned = -1; }
    }
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
    h->run.stream = h->stream;
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
    CHK(alloc_inner(h, h->opt.precision, uses_dc(h)));
    Exec ex{h->stream, nullptr, &h->run.prof};
    if (h->opt.precision == MGWR_FP64) {
        Hier H = plain_hier(h, f, g, u);
        std::vector<Task> ts{Task{&H, (int)h->lv.size() - 1}};
        for (int s = 0; s < sweeps; ++s) CHK(sweep(ex, ts));
        return MGWR_OK;
    }
    // the refinement precisions: the inner hierarchy's kernels on its split
    // storage, f and u reordered into it and u back
    Hier H = inner_hier(h, h->opt.precision);
    H.g = g;
    CHK(enter_inner(ex, H, f, u));
    std::vector<Task> ts{Task{&H, (int)h->lv.size() - 1}};
    for (int s = 0; s < sweeps; ++s) CHK(sweep(ex, ts));
    return leave_inner(ex, H, u);
}

int mgwr_residual(mgwr_t h, const double *f, const double *g, const double *u, double *r, double *norms)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    CHK(check_ptr(r, "r"));
    CHK(set_device(h));
    Exec ex{h->stream, nullptr, &h->run.prof};
    std::vector<FineRes> v{FineRes{h, f, g, u, nullptr, false, norms ? h->run.norms_dev : nullptr, r}};
    CHK(fine_residuals(ex, v));
    if (norms) {
        CHK(read_norms(h->run));
        norms[0] = h->run.norms_host[0];
        norms[1] = h->run.norms_host[1];
    }
    return MGWR_OK;
}

int mgwr_vcycle(mgwr_t h, const double *f, const double *g, double *u)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    CHK(set_device(h));
    CHK(alloc_inner(h, h->opt.precision, uses_dc(h)));
    Exec ex{h->stream, nullptr, &h->run.prof};
    if (h->opt.precision == MGWR_FP64) {
        Hier H = plain_hier(h, f, g, u);
        std::vector<Task> ts{Task{&H, (int)h->lv.size() - 1}};
        return cycle(ex, ts);
    }
    Hier H = inner_hier(h, h->opt.precision);
    H.g = g;
    CHK(enter_inner(ex, H, f, u));
    std::vector<Task> ts{Task{&H, (int)h->lv.size() - 1}};
    CHK(cycle(ex, ts));
    return leave_inner(ex, H, u);
}

int mgwr_solve(mgwr_t h, const double *f, const double *g, double *u, double tol, mgwr_info *info)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(f, "f"));
    CHK(check_ptr(u, "u"));
    if (!(tol >= 0.0)) return fail(MGWR_EINVAL, "tol must be >= 0");
    CHK(set_device(h));
    h->run.stream = h->stream;
    std::vector<mgwr_ctx *> hs{h};
    return solve_group(h->run, hs, &f, &g, &u, tol, info);
}

int mgwr_autotune(mgwr_t h)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(set_device(h));
    h->run.stream = h->stream;
    std::vector<mgwr_ctx *> hs{h};
    return autotune_group(h->run, hs);
}

int mgwr_get_tuning(mgwr_t h, mgwr_tuning *t)
{
    if (!h || !t) return fail(MGWR_EINVAL, "NULL argument");
    tuning_out(h, t);
    return MGWR_OK;
}

int mgwr_set_tuning(mgwr_t h, const mgwr_tuning *t)
{
    if (!h || !t) return fail(MGWR_EINVAL, "NULL argument");
    if (t->levels != (int)h->lv.size()) return fail(MGWR_EINVAL, "the tuning has %d levels, the handle %d", t->levels,
                                                    (int)h->lv.size());
    for (int m = 0; m < 2; ++m)
        if (t->variant[m] < -1 || t->variant[m] > 1) return fail(MGWR_EINVAL, "variant must be -1, 0 or 1");
    for (int m = 0; m < 3; ++m)
        if (t->split_target[m] < 0) return fail(MGWR_EINVAL, "split_target must be >= 0");
    for (int l = 0; l < t->levels; ++l) {
        if (t->dc_block[l] < 0 || t->dc_block[l] % 128 != 0)
            return fail(MGWR_EINVAL, "dc_block must be 0 or a multiple of 128");
        if (t->fft[l] != 0 && t->fft[l] != 1) return fail(MGWR_EINVAL, "fft must be 0 or 1");
    }
    h->tune.kn[GM_F64].variant = t->variant[0];
    h->tune.kn[GM_F32].variant = t->variant[1];
    for (int m = 0; m < 3; ++m) h->tune.kn[m].split_target = t->split_target[m];
    for (int l = 0; l < t->levels; ++l) {
        h->lv[l].dc_tuned = t->dc_block[l];
        h->lv[l].fft_tuned = t->fft[l];
    }
    h->tune.ms_default = t->ms_default;
    h->tune.ms_tuned = t->ms_tuned;
    h->tune.tuned = true;
    clear_programs(h->run);   // recorded programs follow the old choices
    return MGWR_OK;
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
    const int mode = (precision == MGWR_MIXED_FP32) ? GM_F32 : (precision == MGWR_MIXED_BF16X3) ? GM_BF16X3 : GM_F64;
    GemmArgs a = gemm_base(h, mode);
    a.M = h->M; a.P = P; a.K = h->M; a.off = 0; a.coef = coef; a.epi = EPI_STORE;
    a.ea.out = C; a.ea.ldo = ldc;
    Exec ex{h->stream, nullptr, &h->run.prof};
    if (mode == GM_F64) {
        a.B = B; a.ldb = ldb;
        if (fft_for(h, which < 0 ? (int)h->lv.size() - 1 : which))
            set_fft(h, a, which < 0 ? h->spec_tm : h->lv[which].spec_inv);
        return run_gemms(ex, {a}, which);
    }
    // the FFT route in FP32 reads the FP64 operand itself
    const int lev = which < 0 ? (int)h->lv.size() - 1 : which;
    if (fft_for(h, lev, mode)) {
        a.B = B; a.ldb = ldb;
        set_fft32(h, a, which < 0 ? h->spec32_tm : h->lv[which].spec32_inv, true);
        return run_gemms(ex, {a}, which);
    }
    // FP32 / split-BF16 operands are built in temporaries (test path)
    std::vector<void *> tmp;
    int rc = [&]() -> int {
        if (mode == GM_F32) {
            float *b32 = nullptr;
            CHK(dmalloc(tmp, (void **)&b32, sizeof(float) * (size_t)h->M * P));
            HIPCHK(launch_operand({OperandArgs{1, h->M, h->M, P, B, ldb, b32, nullptr, P, nullptr, 0.0}}, nullptr,
                                  h->stream));
            a.B = b32; a.ldb = P;
        } else {
            const long ldp = packed_ld(P);
            uint16_t *hi = nullptr, *lo = nullptr;
            const size_t bytes = sizeof(uint16_t) * (size_t)h->Mpad * ldp;
            CHK(dmalloc(tmp, (void **)&hi, bytes));
            CHK(dmalloc(tmp, (void **)&lo, bytes));
            HIPCHK(launch_operand({OperandArgs{2, h->M, h->Mpad, P, B, ldb, hi, lo, ldp, nullptr, 0.0}}, nullptr,
                                  h->stream));
            a.Bhi = hi; a.Blo = lo; a.ldb = ldp;
        }
        return run_gemms(ex, {a}, which);
    }();
    // the temporaries are freed only after the stream is done with them
    const hipError_t se = hipStreamSynchronize(h->stream);
    free_list(tmp);
    if (rc >= 0 && se != hipSuccess) return fail(MGWR_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(se));
    return rc;
}

int mgwr_toeplitz_apply_static(mgwr_t h, int which, int precision, const double *B, int ldb, int P, double *C,
                               int ldc)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(check_ptr(B, "B"));
    CHK(check_ptr(C, "C"));
    if (which < -1 || which >= (int)h->lv.size()) return fail(MGWR_EINVAL, "bad level %d", which);
    if (P < 1 || ldb < P || ldc < P) return fail(MGWR_EINVAL, "need 1 <= P <= ldb, ldc");
    if (precision < MGWR_FP64 || precision > MGWR_FP64_REFINED) return fail(MGWR_EINVAL, "bad precision");
    CHK(set_device(h));
    if (!h->scratch) CHK(static_scratch(h->device, &h->scratch));
    char *S = (char *)h->scratch;
    const size_t cap = MGWR_STATIC_SCRATCH_BYTES;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const ToepCoef *coef = which < 0 ? &h->tm : &h->lv[which].inv;
    const int lev = which < 0 ? (int)h->lv.size() - 1 : which;
    const int mode = (precision == MGWR_MIXED_FP32) ? GM_F32 : (precision == MGWR_MIXED_BF16X3) ? GM_BF16X3 : GM_F64;
    const long M = h->M;
    GemmArgs a = gemm_base(h, mode);
    a.M = h->M; a.P = P; a.K = h->M; a.off = 0; a.coef = coef; a.epi = EPI_STORE;
    a.ea.out = C; a.ea.ldo = ldc;
    a.part = nullptr; a.part_cap = 0;
    if (mode == GM_F64 ? fft_for(h, lev) : fft_for(h, lev, mode)) {
        // the two work arrays in the two halves; columns beyond what they
        // hold are transformed in chunks
        const size_t half = cap / 2 / 256 * 256, csz = (mode == GM_F64) ? 16 : 8;
        if ((size_t)h->fft_L * csz > half)
            return fail(MGWR_EINVAL, "FFT route: one column pair needs %zu bytes of work array, more than half of "
                        "the %zu-byte static scratch", (size_t)h->fft_L * csz, cap);
        a.B = B; a.ldb = ldb;
        if (mode == GM_F64) set_fft(h, a, which < 0 ? h->spec_tm : h->lv[which].spec_inv);
        else set_fft32(h, a, which < 0 ? h->spec32_tm : h->lv[which].spec32_inv, true);
        a.fft_buf0 = S; a.fft_buf1 = S + half; a.fft_buf_cap = half;
    } else {
        size_t used = 0;
        if (mode == GM_F64) {
            a.B = B; a.ldb = ldb;
        } else if (mode == GM_F32) {
            used = up(sizeof(float) * (size_t)M * P);
            if (used > cap)
                return fail(MGWR_EINVAL, "FP32 operand of %zu bytes exceeds the %zu-byte static scratch", used, cap);
            HIPCHK(launch_operand({OperandArgs{1, h->M, h->M, P, B, ldb, S, nullptr, P, nullptr, 0.0}}, nullptr,
                                  h->stream));
            a.B = S; a.ldb = P;
        } else {
            const long ldp = packed_ld(P);
            const size_t one = up(sizeof(uint16_t) * (size_t)h->Mpad * ldp);
            used = 2 * one;
            if (used > cap)
                return fail(MGWR_EINVAL, "split-BF16 operand of %zu bytes exceeds the %zu-byte static scratch", used,
                            cap);
            HIPCHK(launch_operand({OperandArgs{2, h->M, h->Mpad, P, B, ldb, S, S + one, ldp, nullptr, 0.0}}, nullptr,
                                  h->stream));
            a.Bhi = S; a.Blo = S + one; a.ldb = ldp;
        }
        // split-K partials in the rest (at most what the handle's own buffer
        // holds, so that the launch geometry is the one mgwr_toeplitz_apply uses)
        a.part_cap = std::min(h->part_cap, cap - used);
        a.part = a.part_cap > 0 ? S + used : nullptr;
    }
    HIPCHK(launch_toep_gemm({a}, nullptr, h->stream));
    return MGWR_OK;
}

int mgwr_profile_enable(mgwr_t h, int on)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(set_device(h));
    CHK(h->run.prof.resolve(h->stream));
    if (on) h->run.prof.records.clear();
    h->run.prof.on = on != 0;
    return MGWR_OK;
}

int mgwr_profile_count(mgwr_t h)
{
    if (!h) return fail(MGWR_EINVAL, "NULL handle");
    CHK(set_device(h));
    CHK(h->run.prof.resolve(h->stream));
    return (int)h->run.prof.records.size();
}

int mgwr_profile_get(mgwr_t h, int i, mgwr_kernel_record *rec)
{
    if (!h || !rec) return fail(MGWR_EINVAL, "NULL argument");
    CHK(h->run.prof.resolve(h->stream));
    if (i < 0 || i >= (int)h->run.prof.records.size()) return fail(MGWR_EINVAL, "record %d out of range", i);
    *rec = h->run.prof.records[i];
    return MGWR_OK;
}

const char *mgwr_kernel_name(int kernel)
{
    static thread_local std::string name;
    const int kind = (kernel >> 8) & 15, mode = (kernel >> 4) & 15, epi = kernel & 15;
    const std::string m = std::to_string(mode), e = std::to_string(epi);
    switch (kind) {
    case 0: name = "k_toep_narrow<" + m + ", " + e + ">"; break;
    case 1: name = "k_toep_wide<" + m + ", " + e + ", 0>"; break;
    case 2: name = "k_toep_wide<" + m + ", " + e + ", 1>"; break;
    case 4: name = std::string(mode == 0 ? "k_fft_pass<double> (FFT route, epilogue " : "k_fft_pass<float> (FFT route, epilogue ") + e + ")"; break;
    case 5: name = "k_fft_chip<double> (FFT route on chip, epilogue " + e + ")"; break;
    default: name = "k_toep_bf16x3<" + e + ">"; break;
    }
    return name.c_str();
}

// ---------------------------------------------------------------------------
// Batches: one hierarchy per problem; every stage is one launch over all
// problems that are still iterating.
int mgwr_batch_create(int count, const int *N, const int *M, const double *alpha, const double *T, int dims,
                      const mgwr_options *opts, mgwr_batch_t *out)
{
    if (!out) return fail(MGWR_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (count < 1 || !N || !M || !alpha || !T) return fail(MGWR_EINVAL, "bad batch description");
    mgwr_batch_ctx *b = new mgwr_batch_ctx();
    auto undo = [&](int rc) {
        std::string msg = g_err;
        for (auto x : b->hs) mgwr_destroy(x);
        release_runner(b->run);
        delete b;
        g_err = msg;
        return rc;
    };
    for (int i = 0; i < count; ++i) {
        mgwr_t h = nullptr;
        int rc = mgwr_create_ex(N[i], M[i], alpha[i], T[i], dims, opts, &h);
        if (rc < 0) {
            g_err = "problem " + std::to_string(i) + ": " + g_err;
            return undo(rc);
        }
        b->hs.push_back(h);
    }
    int rc = init_runner(b->run, count);
    if (rc < 0) return undo(rc);
    b->run.graphs = b->hs[0]->opt.graph != 0;
    *out = b;
    return MGWR_OK;
}

int mgwr_batch_set_stream(mgwr_batch_t b, void *hip_stream)
{
    if (!b) return fail(MGWR_EINVAL, "NULL batch");
    b->run.stream = (hipStream_t)hip_stream;
    for (auto h : b->hs) mgwr_set_stream(h, hip_stream);
    return MGWR_OK;
}

int mgwr_batch_solve(mgwr_batch_t b, const double *const *f, const double *const *g, double *const *u,
                     double tol, mgwr_info *infos)
{
    if (!b || !f || !u) return fail(MGWR_EINVAL, "NULL argument");
    if (!(tol >= 0.0)) return fail(MGWR_EINVAL, "tol must be >= 0");
    for (size_t i = 0; i < b->hs.size(); ++i) {
        if (check_ptr(f[i], "f[i]") < 0 || check_ptr(u[i], "u[i]") < 0)
            return fail(MGWR_EINVAL, "problem %zu: f and u must be non-NULL and 8-byte aligned", i);
    }
    CHK(set_device(b->hs[0]));
    return solve_group(b->run, b->hs, f, g, u, tol, infos);
}

int mgwr_batch_autotune(mgwr_batch_t b)
{
    if (!b) return fail(MGWR_EINVAL, "NULL batch");
    CHK(set_device(b->hs[0]));
    return autotune_group(b->run, b->hs);
}

int mgwr_batch_get_tuning(mgwr_batch_t b, int i, mgwr_tuning *t)
{
    if (!b || !t || i < 0 || i >= (int)b->hs.size()) return fail(MGWR_EINVAL, "bad argument");
    tuning_out(b->hs[i], t);
    return MGWR_OK;
}

int mgwr_batch_profile_enable(mgwr_batch_t b, int on)
{
    if (!b) return fail(MGWR_EINVAL, "NULL batch");
    CHK(b->run.prof.resolve(b->run.stream));
    if (on) b->run.prof.records.clear();
    b->run.prof.on = on != 0;
    return MGWR_OK;
}

int mgwr_batch_profile_count(mgwr_batch_t b)
{
    if (!b) return fail(MGWR_EINVAL, "NULL batch");
    CHK(b->run.prof.resolve(b->run.stream));
    return (int)b->run.prof.records.size();
}

int mgwr_batch_profile_get(mgwr_batch_t b, int i, mgwr_kernel_record *rec)
{
    if (!b || !rec) return fail(MGWR_EINVAL, "NULL argument");
    CHK(b->run.prof.resolve(b->run.stream));
    if (i < 0 || i >= (int)b->run.prof.records.size()) return fail(MGWR_EINVAL, "record %d out of range", i);
    *rec = b->run.prof.records[i];
    return MGWR_OK;
}

int mgwr_batch_destroy(mgwr_batch_t b)
{
    if (!b) return MGWR_OK;
    if (b->run.stream) (void)hipStreamSynchronize(b->run.stream);
    release_runner(b->run);
    for (auto h : b->hs) mgwr_destroy(h);
    delete b;
    return MGWR_OK;
}

}  // extern "C"
