// Waveform relaxation FAS for the nonlinear problem of Section 7:
//   D_t^alpha u = (D(u) u_x)_x + c u_x + f on (0, 1), zero initial and
//   boundary values, D(u) = 1 + q u^2 (q = 1 in the paper).
// Discretisation: the L1 scheme in time (lower-triangular Toeplitz T_M with
// first column r); diffusion with the half-point coefficients
// a_{n+-1/2} = (D(u_{n+-1}) + D(u_n)) / 2; the convection term upwinded
// (c >= 0 carries information from the right: forward difference).
// Solver: FAS V(nu1, nu2) cycles over the space hierarchy N_l = 2^(l+1) - 1;
// smoother: red-black nonlinear Gauss-Seidel in which a point's whole time
// line is solved with its neighbours fixed, level by level (T_M is lower
// triangular) by Newton's method; full weighting restricts the residual and
// the solution, linear interpolation carries the coarse correction.
//
// Points are numbered n = 1..N in space (array index n - 1), rows m = 0..M-1
// hold t_{m+1}; colour 0 is even n, colour 1 odd n (the coarse points are
// the even ones).  The smoother gives one wave to each point of a colour:
// the time lines are sequential, the points of a colour independent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mgwr.h"
#include "mgwr_internal.h"

namespace {

constexpr int kNlThreads = 256;
constexpr int kNlMaxM = 4096;   // 2 M doubles of LDS per smoother block
// From this many time levels the residual's T_M u runs on the Toeplitz
// product kernels; below, the per-unknown history sum is faster (N = 255:
// 0.015 ms against 0.040 ms for the product at M = 256, whose few tiles
// leave the GPU mostly idle)
constexpr int kNlProductMinM = 1024;

__device__ inline double nl_D(double q, double v) { return 1.0 + q * v * v; }

// Value of point n (1-based) of a row, zero outside 1..N (Dirichlet).
__device__ inline double nl_at(const double *row, int N, int n) { return (n >= 1 && n <= N) ? row[n - 1] : 0.0; }

// Half-sweep of one colour: the wave (one 64-lane block) of point n solves,
// for m = 0..M-1,
//   r_1 v + sum_{j<m} r_{m-j+1} u_{n,j} - [a+(v)(u_{n+1} - v) - a-(v)(v - u_{n-1})] / h^2
//     - c (u_{n+1} - v) / h = f_{n,m}
// for v = u_{n,m} by Newton's method from the current value.  The time line
// is taken 64 levels at a time, lane L holding level m0 + L: its neighbours,
// f, its old value and its history sum.  At a block's start each lane sums
// the history of the levels before the block; every level solved inside the
// block is then added into the sums of the later lanes, so each level's
// history is complete in its own lane when its turn comes (the same terms in
// the same order as the plain sum over j) and the chain along time holds no
// reduction, only reads of lane k's registers.  The new time line and the
// coefficients are kept in LDS (2 M doubles).
__device__ inline double nl_lane(double x, int k)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(64) void k_nl_sweep(int N, int M, double h, double c, double q, const double *r,
                                                 int colour, const double *f, double *u)
{
    extern __shared__ double lds[];
    double *rs = lds, *tl = lds + M;
    const int lane = threadIdx.x;
    const int n = (colour == 0 ? 2 : 1) + 2 * (int)blockIdx.x;   // the grid holds the colour's points only
    for (int j = lane; j < M; j += 64) rs[j] = r[j];
    __syncthreads();
    const double ih2 = 1.0 / (h * h), ch = c / h, r0 = rs[0];
    for (int m0 = 0; m0 < M; m0 += 64) {
        const int mine = m0 + lane;
        const bool live = mine < M;
        double cul = 0.0, cur = 0.0, cfm = 0.0, cv = 0.0, acc = 0.0;
        if (live) {
            const double *row = u + (size_t)mine * N;
            cul = nl_at(row, N, n - 1);
            cur = nl_at(row, N, n + 1);
            cfm = f[(size_t)mine * N + (n - 1)];
            cv = row[n - 1];
            for (int j = 0; j < m0; ++j) acc += rs[mine - j] * tl[j];   // mine - j in 1..M-1
        }
        const int kend = min(64, M - m0);
        double vmine = cv;
        for (int k = 0; k < kend; ++k) {
            const int d = lane - k;
            const double w = (d > 0 && live) ? rs[d] : 0.0;   // d <= mine < M
            const double hist = nl_lane(acc, k), ul = nl_lane(cul, k), ur = nl_lane(cur, k), fm = nl_lane(cfm, k);
            double v = nl_lane(cv, k);
            for (int it = 0; it < 50; ++it) {
                const double ap = 0.5 * (nl_D(q, ur) + nl_D(q, v)), am = 0.5 * (nl_D(q, ul) + nl_D(q, v));
                const double g = r0 * v + hist - (ap * (ur - v) - am * (v - ul)) * ih2 - ch * (ur - v) - fm;
                const double dg = r0 + (ap + am - q * v * (ur - v) + q * v * (v - ul)) * ih2 + ch;
                const double dv = g / dg;
                v -= dv;
                if (!(fabs(dv) > 1e-15 * (1.0 + fabs(v)))) break;   // converged (or not finite)
            }
            if (lane == k) vmine = v;
            if (d > 0) acc += w * v;
        }
        if (live) {
            tl[mine] = vmine;
            u[(size_t)mine * N + (n - 1)] = vmine;
        }
        __syncthreads();   // the block's levels are in tl before the next block's history sums
    }
}

// out = sf f + sn N(u) + add (f, add may be null): sf = 1, sn = -1 is the
// residual; sf = 0, sn = 1, add = restricted residual the coarse FAS
// right-hand side.  The time-fractional part T_M u (the causal product with
// first column r) is tu, computed before by the FP64 Toeplitz product
// kernels, or (tu null: short time lines) summed here per unknown.
__global__ void k_nl_apply(int N, int M, double h, double c, double q, const double *r, const double *tu,
                           const double *u, const double *f, double sf, double sn, const double *add, double *out)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * N) return;
    const int m = (int)(e / N), n = (int)(e - (long)m * N) + 1;
    double s = 0.0;
    if (tu) {   // a launch-wide choice
        s = tu[e];
    } else {
        // the history sum in order of j, its loads issued eight at a time so
        // that they are in flight together rather than one after another
        const double *col = u + (n - 1);
        int j = 0;
        for (; j + 8 <= m + 1; j += 8) {
            double x[8], w[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                x[t] = col[(size_t)(j + t) * N];
                w[t] = r[m - j - t];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) s += w[t] * x[t];
        }
        for (; j <= m; ++j) s += r[m - j] * col[(size_t)j * N];
    }
    const double *row = u + (size_t)m * N;
    const double uc = row[n - 1], ul = nl_at(row, N, n - 1), ur = nl_at(row, N, n + 1);
    const double ap = 0.5 * (nl_D(q, ur) + nl_D(q, uc)), am = 0.5 * (nl_D(q, ul) + nl_D(q, uc));
    s -= (ap * (ur - uc) - am * (uc - ul)) / (h * h);
    s -= c * (ur - uc) / h;
    double v = sn * s;
    if (f) v += sf * f[e];
    if (add) v += add[e];
    out[e] = v;
}

// Full weighting [1 2 1] / 4 to the coarse grid (coarse J on fine 2J), into
// dst and, when dst2 is not null, into dst2 as well.
__global__ void k_nl_restrict(int Nf, int M, const double *src, double *dst, double *dst2)
{
    const int Nc = (Nf - 1) / 2;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * Nc) return;
    const int m = (int)(e / Nc), J = (int)(e - (long)m * Nc) + 1;
    const double *row = src + (size_t)m * Nf;
    const double v = 0.25 * (nl_at(row, Nf, 2 * J - 1) + 2.0 * nl_at(row, Nf, 2 * J) + nl_at(row, Nf, 2 * J + 1));
    dst[e] = v;
    if (dst2) dst2[e] = v;
}

// uf += linear interpolation of (uc - uc0), zero coarse boundary values.
__global__ void k_nl_prolong_diff(int Nc, int M, const double *uc, const double *uc0, double *uf)
{
    const int Nf = 2 * Nc + 1;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)M * Nf) return;
    const int m = (int)(e / Nf), n = (int)(e - (long)m * Nf) + 1;
    const double *a = uc + (size_t)m * Nc, *b = uc0 + (size_t)m * Nc;
    auto d = [&](int J) { return (J >= 1 && J <= Nc) ? a[J - 1] - b[J - 1] : 0.0; };
    uf[e] += (n % 2 == 0) ? d(n / 2) : 0.5 * (d((n - 1) / 2) + d((n + 1) / 2));
}

// out[0] = max |x_i| over n values (a NaN anywhere makes it NaN); one block
// of kNlMaxThreads threads.
constexpr int kNlMaxThreads = 1024;

__device__ inline double nl_absmax(double a, double v)
{
    v = fabs(v);
    return (v > a || v != v) ? v : a;
}

__global__ __launch_bounds__(kNlMaxThreads) void k_nl_maxabs(long n, const double *x, double *out)
{
    __shared__ double s[kNlMaxThreads];
    double a = 0.0;
    // whole chunks of eight loads per thread, issued together (the maximum
    // does not depend on the order), then the tail one load at a time
    constexpr long chunk = 8L * kNlMaxThreads;
    long i0 = 0;
    for (; i0 + chunk <= n; i0 += chunk) {
        double v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = x[i0 + (long)t * kNlMaxThreads + threadIdx.x];
#pragma unroll
        for (int t = 0; t < 8; ++t) a = nl_absmax(a, v[t]);
    }
    for (long i = i0 + threadIdx.x; i < n; i += kNlMaxThreads) a = nl_absmax(a, x[i]);
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = kNlMaxThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = s[threadIdx.x + w];
            if (o > s[threadIdx.x] || o != o) s[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

struct NlLevel {
    int N = 0;
    double h = 0.0;
    double *u = nullptr, *f = nullptr, *res = nullptr, *uc0 = nullptr;
};

struct NlSolver {
    int M = 0, nu1 = 0, nu2 = 1, first = 1;
    double c = 1.0, q = 1.0;
    const double *r = nullptr;   // device, M coefficients
    mgwr::ToepCoef tc;           // the same, for the product kernels
    double *tu = nullptr;        // device, [M][N of the finest level]: T_M u of the level being applied
                                 // (nullptr: the residual sums the history itself)
    double *part = nullptr;      // split-K partials of that product
    size_t part_cap = 0;
    std::vector<NlLevel> lv;
    hipStream_t s = nullptr;

    static unsigned blocks(long n) { return (unsigned)((n + kNlThreads - 1) / kNlThreads); }

    hipError_t sweep(const NlLevel &L, int colour)
    {
        const int pts = (colour == 0) ? L.N / 2 : (L.N + 1) / 2;
        if (pts <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_nl_sweep, dim3((unsigned)pts), dim3(64), sizeof(double) * 2 * M, s, L.N, M, L.h, c, q,
                           r, colour, (const double *)L.f, L.u);
        return hipGetLastError();
    }
    hipError_t apply(const NlLevel &L, const double *u, const double *f, double sf, double sn, const double *add,
                     double *out)
    {
        if (tu) {
            // long time lines: T_M u by the dense FP64 matrix-core product
            // (O(N M^2) flops near the matrix cores' peak instead of an O(M)
            // loop per unknown), then the rest
            mgwr::GemmArgs a;
            a.mode = mgwr::GM_F64;
            a.M = M; a.P = L.N; a.K = M; a.off = 0; a.coef = &tc;
            a.B = u; a.ldb = L.N;
            a.part = part; a.part_cap = part_cap;
            a.epi = mgwr::EPI_STORE; a.ea.out = tu; a.ea.ldo = L.N;
            hipError_t e = mgwr::launch_toep_gemm({a}, nullptr, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_nl_apply, dim3(blocks((long)M * L.N)), dim3(kNlThreads), 0, s, L.N, M, L.h, c, q, r,
                           (const double *)tu, u, f, sf, sn, add, out);
        return hipGetLastError();
    }
    hipError_t cycle(int l)
    {
        NlLevel &L = lv[l];
        if (l == 0) return sweep(L, 1);   // one point (n = 1): its exact time-line solve
        hipError_t e = hipSuccess;
        for (int i = 0; i < nu1 && e == hipSuccess; ++i) {
            e = sweep(L, first);
            if (e == hipSuccess) e = sweep(L, 1 - first);
        }
        if (e != hipSuccess) return e;
        NlLevel &C = lv[l - 1];
        const long nc = (long)M * C.N;
        if ((e = apply(L, L.u, L.f, 1.0, -1.0, nullptr, L.res)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_nl_restrict, dim3(blocks(nc)), dim3(kNlThreads), 0, s, L.N, M, (const double *)L.res,
                           C.res, (double *)nullptr);
        // coarse start R u, kept in uc0 for the correction
        hipLaunchKernelGGL(k_nl_restrict, dim3(blocks(nc)), dim3(kNlThreads), 0, s, L.N, M, (const double *)L.u,
                           C.uc0, C.u);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // coarse right-hand side N_c(R u) + R (f - N(u))
        if ((e = apply(C, C.uc0, nullptr, 0.0, 1.0, C.res, C.f)) != hipSuccess) return e;
        if ((e = cycle(l - 1)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_nl_prolong_diff, dim3(blocks((long)M * L.N)), dim3(kNlThreads), 0, s, C.N, M,
                           (const double *)C.u, (const double *)C.uc0, L.u);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int i = 0; i < nu2 && e == hipSuccess; ++i) {
            e = sweep(L, first);
            if (e == hipSuccess) e = sweep(L, 1 - first);
        }
        return e;
    }
};

int nl_fail(int code, const char *msg) { return mgwr::set_error(code, msg); }

// One problem of a FAS solve: its hierarchy, coefficients, stream and state.
struct NlProblem {
    NlSolver S;
    double *dmax = nullptr;
    mgwr_info inf{};
    int it = 0, status = MGWR_OK;
    double r0 = 0.0, rn = 0.0;
    bool done = false;
};

// count problems of the same N and M (alpha, f, u per problem): each on its
// own stream, their cycles issued together and their residual norms read
// once per iteration, so the problems' kernels overlap on the GPU.
int fas_solve(int count, int N, int M, const double *alphas, double T, double c, double q, int nu1, int nu2,
              int first_colour, const double *const *f, double *const *u, double tol, int maxit, void *stream,
              mgwr_info *infos)
{
    int k = 0;
    while (((1 << (k + 1)) - 1) < N && k < 30) ++k;
    if (count < 1) return nl_fail(MGWR_EINVAL, "count must be >= 1");
    if (N < 1 || ((1 << (k + 1)) - 1) != N) return nl_fail(MGWR_EINVAL, "N must be 2^k - 1");
    if (M < 1 || M > kNlMaxM) return nl_fail(MGWR_EINVAL, "M must be in 1..4096 (the smoother keeps a time line in LDS)");
    if ((long)M * N > (1L << 30)) return nl_fail(MGWR_EINVAL, "M N too large");
    if (!alphas || !f || !u) return nl_fail(MGWR_EINVAL, "alpha, f and u must not be NULL");
    for (int i = 0; i < count; ++i) {
        if (!(alphas[i] > 0.0 && alphas[i] <= 1.0)) return nl_fail(MGWR_EINVAL, "alpha must be in (0, 1]");
        if (!f[i] || !u[i]) return nl_fail(MGWR_EINVAL, "f and u must not be NULL");
    }
    if (!(T > 0.0) || !std::isfinite(T)) return nl_fail(MGWR_EINVAL, "T must be positive");
    if (!(c >= 0.0) || !std::isfinite(c)) return nl_fail(MGWR_EINVAL, "c must be >= 0 (upwind direction)");
    if (!(q >= 0.0) || !std::isfinite(q)) return nl_fail(MGWR_EINVAL, "q must be >= 0 (D(u) = 1 + q u^2 > 0)");
    if (nu1 < 0 || nu2 < 0 || nu1 + nu2 < 1) return nl_fail(MGWR_EINVAL, "nu1, nu2 >= 0 with nu1 + nu2 >= 1");
    if (first_colour != 0 && first_colour != 1) return nl_fail(MGWR_EINVAL, "first_colour must be 0 or 1");
    if (!(tol > 0.0) || maxit < 0) return nl_fail(MGWR_EINVAL, "tol must be > 0 and maxit >= 0");

    std::vector<std::vector<double>> rh(count, std::vector<double>(M));
    for (int i = 0; i < count; ++i) {
        double cc = 0.0;
        int rc = mgwr_l1_weights(M, alphas[i], T, &cc, rh[i].data());
        if (rc < 0) return rc;
    }

    const hipStream_t caller = (hipStream_t)stream;
    std::vector<NlProblem> P(count);
    std::vector<void *> mem;
    std::vector<hipStream_t> own;
    hipEvent_t start = nullptr;
    double *hnorm = nullptr;   // pinned: the problems' residual norms
    auto alloc = [&](double **p, long n) -> bool {
        if (hipMalloc((void **)p, sizeof(double) * (size_t)std::max(n, 1L)) != hipSuccess) {
            (void)hipGetLastError();   // reported by the caller; not left for a later launch check
            return false;
        }
        mem.push_back(*p);
        return true;
    };
    auto release = [&]() {
        for (const NlProblem &pb : P) (void)hipStreamSynchronize(pb.S.s);   // nothing may still use them
        for (void *p : mem) (void)hipFree(p);
        for (hipStream_t st : own) (void)hipStreamDestroy(st);
        if (start) (void)hipEventDestroy(start);
        if (hnorm) (void)hipHostFree(hnorm);
    };
    bool ok = hipHostMalloc((void **)&hnorm, sizeof(double) * count) == hipSuccess;
    if (!ok) hnorm = nullptr;
    if (ok && count > 1) ok = hipEventCreateWithFlags(&start, hipEventDisableTiming) == hipSuccess &&
                             hipEventRecord(start, caller) == hipSuccess;
    for (int i = 0; i < count && ok; ++i) {
        NlSolver &S = P[i].S;
        S.M = M; S.nu1 = nu1; S.nu2 = nu2; S.first = first_colour; S.c = c; S.q = q;
        if (count == 1) {
            S.s = caller;
        } else {   // default priority; ordered after the caller's earlier work
            ok = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking) == hipSuccess;
            if (!ok) break;
            own.push_back(S.s);
            ok = hipStreamWaitEvent(S.s, start, 0) == hipSuccess;
        }
        ok = ok && alloc((double **)&S.r, M) && alloc(&P[i].dmax, 1);
        S.tc.n = M;
        S.tc.d64 = (double *)S.r;
        if (ok && M >= kNlProductMinM) {
            size_t part = 0;
            for (int l = 0; l <= k; ++l)
                part = std::max(part, mgwr::splitk_bytes(mgwr::GM_F64, M, (1 << (l + 1)) - 1, M, 0, M,
                                                         mgwr::TileKnobs{}));
            ok = alloc(&S.tu, (long)M * N) && (part == 0 || alloc(&S.part, (long)(part / sizeof(double))));
            S.part_cap = S.part ? part : 0;
        }
        S.lv.resize(k + 1);
        for (int l = 0; l <= k && ok; ++l) {
            NlLevel &L = S.lv[l];
            L.N = (1 << (l + 1)) - 1;
            L.h = 1.0 / (L.N + 1);
            const long n = (long)M * L.N;
            ok = alloc(&L.res, n);
            if (ok && l < k) ok = alloc(&L.u, n) && alloc(&L.f, n) && alloc(&L.uc0, n);
        }
        if (ok) {
            S.lv[k].u = u[i];
            S.lv[k].f = (double *)f[i];
        }
    }
    if (!ok) {
        release();
        return nl_fail(MGWR_ENOMEM, "allocation of the FAS hierarchy or its streams failed");
    }
    const long ntop = (long)M * N;
    hipError_t e = hipSuccess;
    for (int i = 0; i < count && e == hipSuccess; ++i) {
        NlSolver &S = P[i].S;
        e = hipMemcpyAsync((void *)S.r, rh[i].data(), sizeof(double) * M, hipMemcpyHostToDevice, S.s);
        if (e == hipSuccess) e = hipMemsetAsync(u[i], 0, sizeof(double) * ntop, S.s);
    }
    int left = count;
    while (e == hipSuccess && left > 0) {
        // residual norms of the problems still iterating
        for (int i = 0; i < count && e == hipSuccess; ++i) {
            if (P[i].done) continue;
            NlSolver &S = P[i].S;
            NlLevel &top = S.lv[k];
            e = S.apply(top, top.u, top.f, 1.0, -1.0, nullptr, top.res);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(k_nl_maxabs, dim3(1), dim3(kNlMaxThreads), 0, S.s, ntop, (const double *)top.res,
                               P[i].dmax);
            if ((e = hipGetLastError()) != hipSuccess) break;
            e = hipMemcpyAsync(&hnorm[i], P[i].dmax, sizeof(double), hipMemcpyDeviceToHost, S.s);
        }
        for (int i = 0; i < count && e == hipSuccess; ++i)
            if (!P[i].done) e = hipStreamSynchronize(P[i].S.s);
        if (e != hipSuccess) break;
        // stopping tests, then one cycle of each problem still iterating
        for (int i = 0; i < count; ++i) {
            NlProblem &pb = P[i];
            if (pb.done) continue;
            pb.rn = hnorm[i];
            bool stop = false;
            if (!std::isfinite(pb.rn)) {
                pb.status = MGWR_ENONFINITE;
                stop = true;
            } else {
                if (pb.it < 128) pb.inf.hist[pb.it] = pb.rn;
                if (pb.it == 0) pb.r0 = pb.rn;
                if (pb.rn <= tol * pb.r0) stop = true;
                else if (pb.it >= maxit) {
                    pb.status = MGWR_NOT_CONVERGED;
                    stop = true;
                }
            }
            if (stop) {
                pb.done = true;
                --left;
            }
        }
        for (int i = 0; i < count && e == hipSuccess; ++i) {
            if (P[i].done) continue;
            e = P[i].S.cycle(k);
            ++P[i].it;
        }
    }
    release();
    if (e != hipSuccess) return nl_fail(MGWR_EDEVICE, hipGetErrorString(e));
    int worst = MGWR_OK;
    for (int i = 0; i < count; ++i) {
        NlProblem &pb = P[i];
        pb.inf.iters = pb.it;
        pb.inf.status = pb.status;
        pb.inf.r0 = pb.r0;
        pb.inf.rk = pb.rn;
        pb.inf.relres = pb.r0 > 0.0 ? pb.rn / pb.r0 : 0.0;
        pb.inf.mean_factor = (pb.it > 0 && pb.r0 > 0.0) ? std::pow(pb.rn / pb.r0, 1.0 / pb.it) : 0.0;
        if (infos) infos[i] = pb.inf;
        if (pb.status == MGWR_ENONFINITE) worst = MGWR_ENONFINITE;
        else if (pb.status == MGWR_NOT_CONVERGED && worst == MGWR_OK) worst = MGWR_NOT_CONVERGED;
    }
    if (worst == MGWR_ENONFINITE) return nl_fail(MGWR_ENONFINITE, "the residual is not finite");
    return worst;
}

}  // namespace

extern "C" int mgwr_fas_solve(int N, int M, double alpha, double T, double c, double q, int nu1, int nu2,
                              int first_colour, const double *f, double *u, double tol, int maxit, void *stream,
                              mgwr_info *info)
{
    return fas_solve(1, N, M, &alpha, T, c, q, nu1, nu2, first_colour, &f, &u, tol, maxit, stream, info);
}

extern "C" int mgwr_fas_solve_batch(int count, int N, int M, const double *alpha, double T, double c, double q,
                                    int nu1, int nu2, int first_colour, const double *const *f, double *const *u,
                                    double tol, int maxit, void *stream, mgwr_info *infos)
{
    return fas_solve(count, N, M, alpha, T, c, q, nu1, nu2, first_colour, f, u, tol, maxit, stream, infos);
}
