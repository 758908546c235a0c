// HIP kernels for gfx950 (MI355X) of multigrid waveform relaxation for the
// time-fractional heat equation (Gaspar & Rodrigo, arXiv:1608.05400).
//
// Data layout: every grid function of a level is time-major, [M][P] with the
// P points of the level contiguous (x fastest in 2D).  The L1 time operator
// couples only the rows of one column, so one Toeplitz product over all
// columns of a level (or of one colour) is a GEMM whose A operand is the
// lower-triangular Toeplitz matrix generated from its first column.
//
// Toeplitz products (Section 5: the defect needs T_M x per spatial point, the
// smoother solves with T_M + sigma I):
//   * k_toep_wide / k_toep_narrow: FP64 (v_mfma_f64_16x16x4_f64) and FP32
//     (v_mfma_f32_16x16x4_f32).  The Toeplitz tile is never stored: the
//     BM + BK - 1 coefficients a tile needs are staged in LDS and every lane
//     gathers its A element t[i - k] from that window.
//   * k_toep_bf16x3: split-BF16 with three v_mfma_f32_16x16x32_bf16 passes
//     (hi*hi + hi*lo + lo*hi) and FP32 accumulation.  The Toeplitz operand is
//     materialised once per coefficient vector as a table of MFMA-ready
//     fragments (one per diagonal offset multiple of 16) and staged in LDS.
// Everything else (colour right-hand sides, residual stencils, transfers,
// norms, precision updates) is bandwidth bound and written for coalescing.
#include "mgwr_internal.h"

namespace mgwr {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// BF16 helpers: round-to-nearest-even of a finite float, and back.
__device__ inline uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// Stencils of the negative Laplacian (Section 2: 3-point; Section 6: 5-point)
// with zero Dirichlet values, on one time row U of a level with n points/dim.
template <typename S>
__device__ inline double nbr_sum(const S *U, int dims, int n, int p)
{
    if (dims == 1) {
        double s = 0.0;
        if (p > 0) s += (double)U[p - 1];
        if (p < n - 1) s += (double)U[p + 1];
        return s;
    }
    int x = p % n, y = p / n;
    double s = 0.0;
    if (x > 0) s += (double)U[p - 1];
    if (x < n - 1) s += (double)U[p + 1];
    if (y > 0) s += (double)U[p - n];
    if (y < n - 1) s += (double)U[p + n];
    return s;
}

__device__ inline void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// A_h (hi + lo) at point p as an unevaluated sum (shi + slo) / h^2:
// shi + slo = 2 d hi_p - sum(neighbours of hi) + (same stencil of lo),
// the hi part without rounding error (error-free transformations).
__device__ inline void stencil_dd(const double *H, const double *Lo, int dims, int n, int p,
                                  double &shi, double &slo)
{
    double s = (dims == 1 ? 2.0 : 4.0) * H[p], e, acc = 0.0;
    double lo = (dims == 1 ? 2.0 : 4.0) * Lo[p];
    if (dims == 1) {
        if (p > 0) { two_sum(s, -H[p - 1], s, e); acc += e; lo -= Lo[p - 1]; }
        if (p < n - 1) { two_sum(s, -H[p + 1], s, e); acc += e; lo -= Lo[p + 1]; }
    } else {
        int x = p % n, y = p / n;
        if (x > 0) { two_sum(s, -H[p - 1], s, e); acc += e; lo -= Lo[p - 1]; }
        if (x < n - 1) { two_sum(s, -H[p + 1], s, e); acc += e; lo -= Lo[p + 1]; }
        if (y > 0) { two_sum(s, -H[p - n], s, e); acc += e; lo -= Lo[p - n]; }
        if (y < n - 1) { two_sum(s, -H[p + n], s, e); acc += e; lo -= Lo[p + n]; }
    }
    shi = s;
    slo = acc + lo;
}

// ---------------------------------------------------------------------------
// Epilogue of the Toeplitz products, element (i, p) with product value acc.
// All grid functions are FP64.
template <int EPI>
__device__ inline void epi_apply(const EpiArgs &e, int i, int p, double acc)
{
    if constexpr (EPI == EPI_STORE) {
        e.out[(long)i * e.ldo + p] = acc;
    } else if constexpr (EPI == EPI_SUB) {
        double *o = e.out + (long)i * e.ldo + p;
        *o = *o - acc;
    } else if constexpr (EPI == EPI_SCATTER) {
        e.out[(long)i * e.ldo + colour_point(e.dims, e.n, e.colour, p)] = acc;
    } else if constexpr (EPI == EPI_SMOOTH) {
        // x = t0 b + (history product); b rebuilt from F and the other colour
        // of U, which this half-sweep does not write.
        const int pt = colour_point(e.dims, e.n, e.colour, p);
        const double *Ui = e.out + (long)i * e.ld;
        double b = e.F[(long)i * e.ld + pt] + nbr_sum(Ui, e.dims, e.n, pt) * e.ih2;
        if (e.g) b += e.cd[i] * e.g[pt];
        e.out[(long)i * e.ldo + pt] = e.diag * b + acc;
    } else if constexpr (EPI == EPI_RESID) {
        const double *U = e.U + (long)i * e.ld;
        double rhs = e.F[(long)i * e.ld + p];
        if (e.g) rhs += e.cd[i] * e.g[p];
        double u = U[p];
        double st = (e.dims == 1 ? 2.0 : 4.0) * u - nbr_sum(U, e.dims, e.n, p);
        e.out[(long)i * e.ldo + p] = rhs - e.diag * u - acc - st * e.ih2;
    } else if constexpr (EPI == EPI_RESID_DD) {
        const double *H = e.U + (long)i * e.ld;
        const double *Lo = e.ulo + (long)i * e.ld;
        double rhs = e.F[(long)i * e.ld + p];
        if (e.g) rhs += e.cd[i] * e.g[p];
        double shi, slo;
        stencil_dd(H, Lo, e.dims, e.n, p, shi, slo);
        e.out[(long)i * e.ldo + p] = ((rhs - acc) - shi * e.ih2) - slo * e.ih2;
    }
}

// Kernel parameters (passed by value).
struct KP {
    int M, P, K, off, ncoef;
    int tiles_m, tiles_n;
    const void *coef;          // double* or float* (F64/F32)
    const uint16_t *fhi, *flo; // fragment tables (BF16X3)
    const void *B;
    const uint16_t *Bhi, *Blo;
    long ldb;
    EpiArgs ea;
};

template <int MODE> struct Tr;
template <> struct Tr<GM_F64> {
    using S = double;
    using acc_t = v4d;
    __device__ static acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of accumulator element v of lane (column = lane % 16)
    __device__ static int crow(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Tr<GM_F32> {
    using S = float;
    using acc_t = v4f;
    __device__ static acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int crow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// ---------------------------------------------------------------------------
// Wide Toeplitz product: block tile 128 x 64, 4 waves in 2 x 2, wave tile
// 64 x 32 (4 x 2 MFMA blocks of 16 x 16), K step 16, LDS double buffer.
// Block order: largest row index first (causal products have the most work
// there), so the short tiles fill the tail of the launch.
constexpr int WBM = 128, WBN = 64, WBK = 16, WWIN = WBM + WBK;

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void k_toep_wide(KP kp)
{
    using T = Tr<MODE>;
    using S = typename T::S;
    using acc_t = typename T::acc_t;
    __shared__ S Bs[2][WBK][WBN];
    __shared__ S Ws[2][WWIN];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int t = blockIdx.x;
    const int tm = kp.tiles_m - 1 - t / kp.tiles_n, tn = t % kp.tiles_n;
    const int i0 = tm * WBM, p0 = tn * WBN;
    const S *coef = (const S *)kp.coef;
    const S *B = (const S *)kp.B;

    int kend = min(kp.K, i0 + WBM + kp.off);
    int kbeg = max(0, kp.off + i0 - kp.ncoef + 1);
    kbeg = (kbeg / WBK) * WBK;
    const int nk = (kend > kbeg) ? (kend - kbeg + WBK - 1) / WBK : 0;

    acc_t acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

    const int brow = tid >> 4, bc4 = (tid & 15) * 4;
    S breg[4];
    S wreg = 0;
    auto gload = [&](int k0) {
        int k = k0 + brow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int p = p0 + bc4 + j;
            breg[j] = (k < kp.K && p < kp.P) ? B[(long)k * kp.ldb + p] : (S)0;
        }
        if (tid < WWIN) {
            int s = kp.off + i0 - k0 - (WBK - 1) + tid;
            wreg = (s >= 0 && s < kp.ncoef) ? coef[s] : (S)0;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int j = 0; j < 4; ++j) Bs[buf][brow][bc4 + j] = breg[j];
        if (tid < WWIN) Ws[buf][tid] = wreg;
    };

    if (nk > 0) {
        gload(kbeg);
        sstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload(kbeg + (kt + 1) * WBK);
#pragma unroll
        for (int ks = 0; ks < WBK / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            S a[4], b[2];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = Ws[buf][wm * 64 + 16 * x + (lane & 15) - kr + WBK - 1];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = Bs[buf][kr][wn * 32 + 16 * y + (lane & 15)];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = T::mma(a[x], b[y], acc[x][y]);
        }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int i = i0 + wm * 64 + 16 * x + T::crow(lane, v);
                int p = p0 + wn * 32 + 16 * y + (lane & 15);
                if (i < kp.M && p < kp.P) epi_apply<EPI>(kp.ea, i, p, (double)acc[x][y][v]);
            }
}

// ---------------------------------------------------------------------------
// Narrow Toeplitz product for levels with few columns (coarse grids): block
// tile 64 x 16; the four waves split the K range (chunks of 16 rows taken
// round-robin) and their partial tiles are summed in LDS in a fixed order.
constexpr int NBM = 64, NBN = 16, NCH = 16;

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void k_toep_narrow(KP kp)
{
    using T = Tr<MODE>;
    using S = typename T::S;
    using acc_t = typename T::acc_t;
    __shared__ S red[4][NBM * NBN];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int t = blockIdx.x;
    const int tm = kp.tiles_m - 1 - t / kp.tiles_n, tn = t % kp.tiles_n;
    const int i0 = tm * NBM, p0 = tn * NBN;
    const S *coef = (const S *)kp.coef;
    const S *B = (const S *)kp.B;

    int kend = min(kp.K, i0 + NBM + kp.off);
    int kbeg = max(0, kp.off + i0 - kp.ncoef + 1);
    kbeg = (kbeg / NCH) * NCH;
    const int nch = (kend > kbeg) ? (kend - kbeg + NCH - 1) / NCH : 0;

    acc_t acc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) acc[x] = acc_t{0, 0, 0, 0};
    const int pc = p0 + (lane & 15);
    for (int c = wid; c < nch; c += 4) {
        const int k0 = kbeg + c * NCH;
#pragma unroll
        for (int ks = 0; ks < NCH / 4; ++ks) {
            const int k = k0 + 4 * ks + (lane >> 4);
            S b = (k < kp.K && pc < kp.P) ? B[(long)k * kp.ldb + pc] : (S)0;
            S a[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                int s = kp.off + i0 + 16 * x + (lane & 15) - k;
                a[x] = (s >= 0 && s < kp.ncoef) ? coef[s] : (S)0;
            }
#pragma unroll
            for (int x = 0; x < 4; ++x) acc[x] = T::mma(a[x], b, acc[x]);
        }
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wid][(16 * x + T::crow(lane, v)) * NBN + (lane & 15)] = acc[x][v];
    __syncthreads();
    for (int e = tid; e < NBM * NBN; e += 256) {
        int row = e / NBN, col = e % NBN;
        double sum = (double)red[0][e] + (double)red[1][e] + (double)red[2][e] + (double)red[3][e];
        int i = i0 + row, p = p0 + col;
        if (i < kp.M && p < kp.P) epi_apply<EPI>(kp.ea, i, p, sum);
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 Toeplitz product.  Block tile 128 x 128, 4 waves in 2 x 2, wave
// tile 64 x 64 (4 x 4 blocks of 16 x 16), K step 32.  Per K step the block
// stages 8 Toeplitz fragments (hi and lo, 16 KB) from the fragment table and
// the B tile (hi and lo, k8-packed, 16 KB) into LDS (double buffered).
// B must be k8-packed with rows padded to a multiple of 128 and columns to a
// multiple of 128, padding zero.
constexpr int BBM = 128, BBN = 128, BBK = 32;

__device__ inline v8bf as_bf8(uint4 v) { return __builtin_bit_cast(v8bf, v); }

template <int EPI>
__global__ __launch_bounds__(256) void k_toep_bf16x3(KP kp)
{
    __shared__ uint4 As[2][2][8][64];        // [buf][hi/lo][fragment][lane]
    __shared__ uint4 Bs[2][2][4][BBN];       // [buf][hi/lo][k/8][column]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int t = blockIdx.x;
    const int tm = kp.tiles_m - 1 - t / kp.tiles_n, tn = t % kp.tiles_n;
    const int i0 = tm * BBM, p0 = tn * BBN;

    int kend = min(kp.K, i0 + BBM + kp.off);
    int kbeg = max(0, kp.off + i0 - kp.ncoef + 1);
    kbeg = (kbeg / BBK) * BBK;
    const int nk = (kend > kbeg) ? (kend - kbeg + BBK - 1) / BBK : 0;

    v4f acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = v4f{0, 0, 0, 0};

    const uint4 *fh = (const uint4 *)kp.fhi, *fl = (const uint4 *)kp.flo;
    const uint4 *bh = (const uint4 *)kp.Bhi, *bl = (const uint4 *)kp.Blo;
    uint4 ra[4], rb[4];
    auto gload = [&](int k0) {
        const int q0 = (kp.off + i0 - k0) / 16 + kQOff;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int u = tid + 256 * r;
            int hl = u >> 9, a = (u >> 6) & 7, ln = u & 63;
            ra[r] = (hl ? fl : fh)[(long)(q0 + a) * 64 + ln];
            int kg = (u >> 7) & 3, col = u & 127;
            rb[r] = (hl ? bl : bh)[(long)(k0 / 8 + kg) * kp.ldb + p0 + col];
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int u = tid + 256 * r;
            int hl = u >> 9;
            As[buf][hl][(u >> 6) & 7][u & 63] = ra[r];
            Bs[buf][hl][(u >> 7) & 3][u & 127] = rb[r];
        }
    };

    if (nk > 0) {
        gload(kbeg);
        sstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload(kbeg + (kt + 1) * BBK);
        v8bf ah[4], al[4], bhv[4], blv[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            ah[x] = as_bf8(As[buf][0][wm * 4 + x][lane]);
            al[x] = as_bf8(As[buf][1][wm * 4 + x][lane]);
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            bhv[y] = as_bf8(Bs[buf][0][lane >> 4][wn * 64 + 16 * y + (lane & 15)]);
            blv[y] = as_bf8(Bs[buf][1][lane >> 4][wn * 64 + 16 * y + (lane & 15)]);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], bhv[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], blv[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[x], bhv[y], acc[x][y], 0, 0, 0);
            }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int i = i0 + wm * 64 + 16 * x + 4 * (lane >> 4) + v;
                int p = p0 + wn * 64 + 16 * y + (lane & 15);
                if (i < kp.M && p < kp.P) epi_apply<EPI>(kp.ea, i, p, (double)acc[x][y][v]);
            }
}

// ---------------------------------------------------------------------------
template <int MODE, int EPI>
static hipError_t launch_mode_epi(const GemmArgs &a, KP &kp, hipStream_t s)
{
    if constexpr (MODE == GM_BF16X3) {
        kp.tiles_m = (a.M + BBM - 1) / BBM;
        kp.tiles_n = (a.P + BBN - 1) / BBN;
        hipLaunchKernelGGL((k_toep_bf16x3<EPI>), dim3(kp.tiles_m * kp.tiles_n), dim3(256), 0, s, kp);
    } else if (a.P <= 32) {
        kp.tiles_m = (a.M + NBM - 1) / NBM;
        kp.tiles_n = (a.P + NBN - 1) / NBN;
        hipLaunchKernelGGL((k_toep_narrow<MODE, EPI>), dim3(kp.tiles_m * kp.tiles_n), dim3(256), 0, s, kp);
    } else {
        kp.tiles_m = (a.M + WBM - 1) / WBM;
        kp.tiles_n = (a.P + WBN - 1) / WBN;
        hipLaunchKernelGGL((k_toep_wide<MODE, EPI>), dim3(kp.tiles_m * kp.tiles_n), dim3(256), 0, s, kp);
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(const GemmArgs &a, KP &kp, hipStream_t s)
{
    switch (a.epi) {
    case EPI_STORE: return launch_mode_epi<MODE, EPI_STORE>(a, kp, s);
    case EPI_SCATTER: return launch_mode_epi<MODE, EPI_SCATTER>(a, kp, s);
    case EPI_SMOOTH: return launch_mode_epi<MODE, EPI_SMOOTH>(a, kp, s);
    case EPI_RESID: return launch_mode_epi<MODE, EPI_RESID>(a, kp, s);
    case EPI_SUB: return launch_mode_epi<MODE, EPI_SUB>(a, kp, s);
    case EPI_RESID_DD:
        if constexpr (MODE == GM_F64) return launch_mode_epi<MODE, EPI_RESID_DD>(a, kp, s);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_toep_gemm(const GemmArgs &a, hipStream_t s)
{
    if (a.M <= 0 || a.P <= 0) return hipSuccess;
    KP kp{};
    kp.M = a.M; kp.P = a.P; kp.K = a.K; kp.off = a.off; kp.ncoef = a.coef->n;
    kp.B = a.B; kp.Bhi = (const uint16_t *)a.Bhi; kp.Blo = (const uint16_t *)a.Blo; kp.ldb = a.ldb;
    kp.ea = a.ea;
    switch (a.mode) {
    case GM_F64: kp.coef = a.coef->d64; return launch_mode<GM_F64>(a, kp, s);
    case GM_F32: kp.coef = a.coef->d32; return launch_mode<GM_F32>(a, kp, s);
    case GM_BF16X3:
        kp.fhi = a.coef->fhi; kp.flo = a.coef->flo;
        return launch_mode<GM_BF16X3>(a, kp, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Colour right-hand side of the smoother (Section 3, eq. red-black; Section 6,
// eq. red-black_2d): b = f + c d g + (neighbour sum) / h^2 at the points of
// one colour, gathered into a dense panel (the B operand of the product).
template <typename S>
__global__ void k_rhs_panel(int dims, int n, int colour, int M, int Pc, const double *F,
                            const double *U, const double *cd, const double *g, double ih2, S *panel,
                            long ldp)
{
    long P = (dims == 1) ? n : (long)n * n;
    long total = (long)M * Pc;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int k = (int)(e / Pc), j = (int)(e - (long)k * Pc);
        int pt = colour_point(dims, n, colour, j);
        const double *Uk = U + (long)k * P;
        double b = F[(long)k * P + pt] + nbr_sum(Uk, dims, n, pt) * ih2;
        if (g) b += cd[k] * g[pt];
        panel[(long)k * ldp + j] = (S)b;
    }
}

__device__ inline void store_split8(const float *b, uint16_t *hi, uint16_t *lo, long e)
{
    uint16_t h8[8], l8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint16_t hb = f2bf(b[q]);
        h8[q] = hb;
        l8[q] = f2bf(b[q] - bf2f(hb));
    }
    uint4 vh, vl;
    vh.x = h8[0] | ((uint32_t)h8[1] << 16); vh.y = h8[2] | ((uint32_t)h8[3] << 16);
    vh.z = h8[4] | ((uint32_t)h8[5] << 16); vh.w = h8[6] | ((uint32_t)h8[7] << 16);
    vl.x = l8[0] | ((uint32_t)l8[1] << 16); vl.y = l8[2] | ((uint32_t)l8[3] << 16);
    vl.z = l8[4] | ((uint32_t)l8[5] << 16); vl.w = l8[6] | ((uint32_t)l8[7] << 16);
    ((uint4 *)hi)[e] = vh;
    ((uint4 *)lo)[e] = vl;
}

// Same right-hand side as split BF16 hi/lo in the k8-packed layout
// [Mpad/8][ldp][8] (zero outside k < M, j < Pc).  One thread builds the 8
// time rows of one column.
__global__ void k_rhs_panel_packed(int dims, int n, int colour, int M, int Mpad, int Pc,
                                   const double *F, const double *U, const double *cd,
                                   const double *g, double ih2, uint16_t *hi, uint16_t *lo, long ldp)
{
    long P = (dims == 1) ? n : (long)n * n;
    long total = (long)(Mpad / 8) * ldp;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int kg = (int)(e / ldp), j = (int)(e - (long)kg * ldp);
        float b8[8];
        int pt = (j < Pc) ? colour_point(dims, n, colour, j) : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int k = kg * 8 + q;
            double b = 0.0;
            if (k < M && j < Pc) {
                const double *Uk = U + (long)k * P;
                b = F[(long)k * P + pt] + nbr_sum(Uk, dims, n, pt) * ih2;
                if (g) b += cd[k] * g[pt];
            }
            b8[q] = (float)b;
        }
        store_split8(b8, hi, lo, e);
    }
}

__global__ void k_split_bf16(int M, int Mpad, int P, const double *X, uint16_t *hi, uint16_t *lo,
                             long ldp)
{
    long total = (long)(Mpad / 8) * ldp;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int kg = (int)(e / ldp), j = (int)(e - (long)kg * ldp);
        float b8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int k = kg * 8 + q;
            b8[q] = (k < M && j < P) ? (float)X[(long)k * P + j] : 0.0f;
        }
        store_split8(b8, hi, lo, e);
    }
}

__global__ void k_narrow_f32(long n, const double *x, float *y)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

__global__ void k_widen(long n, const float *x, double *y)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

// Full weighting (Section 3; Section 6): coarse node J on fine node 2J,
// weights [1 2 1]/4 (1D) and their tensor product /16 (2D).
__global__ void k_restrict(int dims, int nf, int M, const double *rf, double *rc)
{
    int nc = (nf - 1) / 2;
    long Pc = (dims == 1) ? nc : (long)nc * nc;
    long Pf = (dims == 1) ? nf : (long)nf * nf;
    long total = (long)M * Pc;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int k = (int)(e / Pc);
        long q = e - (long)k * Pc;
        const double *r = rf + (long)k * Pf;
        double v;
        if (dims == 1) {
            int x = 2 * (int)q + 1;
            v = 0.25 * (r[x - 1] + 2.0 * r[x] + r[x + 1]);
        } else {
            int I = (int)(q % nc), J = (int)(q / nc);
            int x = 2 * I + 1, y = 2 * J + 1;
            const double *r0 = r + (long)(y - 1) * nf, *r1 = r + (long)y * nf, *r2 = r + (long)(y + 1) * nf;
            v = (r0[x - 1] + 2.0 * r0[x] + r0[x + 1] + 2.0 * (r1[x - 1] + 2.0 * r1[x] + r1[x + 1])
                 + r2[x - 1] + 2.0 * r2[x] + r2[x + 1]) * (1.0 / 16.0);
        }
        rc[e] = v;
    }
}

// Linear / bilinear interpolation of the coarse correction, added to the fine
// iterate (Section 3; Section 6); coarse values on the boundary are zero.
__device__ inline double coarse_at(const double *e, int nc, int X)  // X: 1-based coarse index
{
    return (X >= 1 && X <= nc) ? e[X - 1] : 0.0;
}

__global__ void k_prolong_add(int dims, int nc, int M, const double *ec, double *uf)
{
    int nf = 2 * nc + 1;
    long Pc = (dims == 1) ? nc : (long)nc * nc;
    long Pf = (dims == 1) ? nf : (long)nf * nf;
    long total = (long)M * Pf;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int k = (int)(e / Pf);
        long p = e - (long)k * Pf;
        const double *c = ec + (long)k * Pc;
        double v;
        if (dims == 1) {
            int nn = (int)p + 1;   // paper numbering
            v = 0.5 * (coarse_at(c, nc, nn / 2) + coarse_at(c, nc, (nn + 1) / 2));
        } else {
            int nn = (int)(p % nf) + 1, ll = (int)(p / nf) + 1;
            int xa = nn / 2, xb = (nn + 1) / 2, ya = ll / 2, yb = (ll + 1) / 2;
            auto at = [&](int X, int Y) -> double {
                return (X >= 1 && X <= nc && Y >= 1 && Y <= nc) ? c[(long)(Y - 1) * nc + (X - 1)] : 0.0;
            };
            v = 0.25 * (at(xa, ya) + at(xb, ya) + at(xa, yb) + at(xb, yb));
        }
        uf[e] += v;
    }
}

__global__ void k_fill(long M, long P, const double *g, double *u)
{
    long total = M * P;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        u[e] = g ? g[e % P] : 0.0;
    }
}

// Deterministic norm partials: each block reduces a fixed contiguous share.
constexpr int kNormThreads = 256;
int norm_partial_blocks(long n)
{
    long b = (n + 8L * kNormThreads - 1) / (8L * kNormThreads);
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

__global__ __launch_bounds__(kNormThreads) void k_norm_partials(long n, const double *x, double *partials)
{
    __shared__ double smax[kNormThreads], ssum[kNormThreads];
    long per = (n + gridDim.x - 1) / gridDim.x;
    long beg = (long)blockIdx.x * per, end = min(n, beg + per);
    double mx = 0.0, sq = 0.0;
    for (long e = beg + threadIdx.x; e < end; e += kNormThreads) {
        double v = x[e];
        double a = fabs(v);
        mx = (a > mx || a != a) ? a : mx;   // keeps a NaN once seen
        sq += v * v;
    }
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = sq;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double a = smax[threadIdx.x + w];
            double m = smax[threadIdx.x];
            smax[threadIdx.x] = (a > m || a != a) ? a : m;
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = smax[0];
        partials[2 * blockIdx.x + 1] = ssum[0];
    }
}

__global__ __launch_bounds__(kNormThreads) void k_norm_final(int nblk, const double *partials, double *out2)
{
    __shared__ double smax[kNormThreads], ssum[kNormThreads];
    double mx = 0.0, sq = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kNormThreads) {
        double a = partials[2 * b];
        mx = (a > mx || a != a) ? a : mx;
        sq += partials[2 * b + 1];
    }
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = sq;
    __syncthreads();
    for (int w = kNormThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double a = smax[threadIdx.x + w];
            double m = smax[threadIdx.x];
            smax[threadIdx.x] = (a > m || a != a) ? a : m;
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[0] = smax[0];
        out2[1] = sqrt(ssum[0]);
    }
}

// (hi, lo) <- (hi, lo) + e as a renormalised double-double (TwoSum, then
// fast renormalisation); with lo == nullptr a plain FP64 add.
__global__ void k_dd_update(long n, const double *e, double *hi, double *lo)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        double d = e[i];
        if (!lo) {
            hi[i] += d;
            continue;
        }
        double s, err;
        two_sum(hi[i], d, s, err);
        double l = lo[i] + err;
        double h2 = s + l;
        lo[i] = l - (h2 - s);
        hi[i] = h2;
    }
}

// FP32 copy and BF16 fragment table of a coefficient vector.
__global__ void k_build_coef(int n, const double *d64, float *d32, int nq, uint16_t *fhi, uint16_t *flo)
{
    long tot = (long)nq * 64 * 8;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot + n;
         e += (long)gridDim.x * blockDim.x) {
        if (e < n) d32[e] = (float)d64[e];
        if (e < tot) {
            int q = (int)(e / 512) - kQOff;
            int ln = (int)((e / 8) % 64), el = (int)(e % 8);
            int s = 16 * q + (ln & 15) - (8 * (ln >> 4) + el);
            float v = (s >= 0 && s < n) ? (float)d64[s] : 0.0f;
            uint16_t h = f2bf(v);
            fhi[e] = h;
            flo[e] = f2bf(v - bf2f(h));
        }
    }
}

// ---------------------------------------------------------------------------
static inline dim3 grid_for(long total, int threads = 256)
{
    long b = (total + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return dim3((unsigned)b);
}

hipError_t launch_rhs_panel(int fmt, int dims, int n, int colour, int M, int Mpad, const double *F,
                            const double *U, const double *cd, const double *g, double ih2,
                            void *panel, void *panel_lo, long ldp, hipStream_t s)
{
    int Pc = colour_count(dims, n, colour);
    if (fmt == 2) {
        long total = (long)(Mpad / 8) * ldp;
        hipLaunchKernelGGL(k_rhs_panel_packed, grid_for(total), dim3(256), 0, s, dims, n, colour, M, Mpad,
                           Pc, F, U, cd, g, ih2, (uint16_t *)panel, (uint16_t *)panel_lo, ldp);
    } else if (fmt == 0) {
        hipLaunchKernelGGL(k_rhs_panel<double>, grid_for((long)M * Pc), dim3(256), 0, s, dims, n, colour,
                           M, Pc, F, U, cd, g, ih2, (double *)panel, ldp);
    } else {
        hipLaunchKernelGGL(k_rhs_panel<float>, grid_for((long)M * Pc), dim3(256), 0, s, dims, n, colour,
                           M, Pc, F, U, cd, g, ih2, (float *)panel, ldp);
    }
    return hipGetLastError();
}

hipError_t launch_operand(int fmt, int M, int Mpad, int P, const double *X, void *out, void *out_lo,
                          long ldp, hipStream_t s)
{
    if (fmt == 2) {
        long total = (long)(Mpad / 8) * ldp;
        hipLaunchKernelGGL(k_split_bf16, grid_for(total), dim3(256), 0, s, M, Mpad, P, X, (uint16_t *)out,
                           (uint16_t *)out_lo, ldp);
    } else {
        long n = (long)M * P;
        hipLaunchKernelGGL(k_narrow_f32, grid_for(n), dim3(256), 0, s, n, X, (float *)out);
    }
    return hipGetLastError();
}

hipError_t launch_widen(long n, const float *x, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_widen, grid_for(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t launch_restrict(int dims, int nf, int M, const double *rf, double *rc, hipStream_t s)
{
    int nc = (nf - 1) / 2;
    long total = (long)M * ((dims == 1) ? nc : (long)nc * nc);
    hipLaunchKernelGGL(k_restrict, grid_for(total), dim3(256), 0, s, dims, nf, M, rf, rc);
    return hipGetLastError();
}

hipError_t launch_prolong_add(int dims, int nc, int M, const double *ec, double *uf, hipStream_t s)
{
    int nf = 2 * nc + 1;
    long total = (long)M * ((dims == 1) ? nf : (long)nf * nf);
    hipLaunchKernelGGL(k_prolong_add, grid_for(total), dim3(256), 0, s, dims, nc, M, ec, uf);
    return hipGetLastError();
}

hipError_t launch_fill(long M, long P, const double *g, double *u, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, grid_for(M * P), dim3(256), 0, s, M, P, g, u);
    return hipGetLastError();
}

hipError_t launch_norm_partials(long n, const double *x, double *partials, int *nblk, hipStream_t s)
{
    int b = norm_partial_blocks(n);
    *nblk = b;
    hipLaunchKernelGGL(k_norm_partials, dim3(b), dim3(kNormThreads), 0, s, n, x, partials);
    return hipGetLastError();
}

hipError_t launch_norm_final(int nblk, const double *partials, double *out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kNormThreads), 0, s, nblk, partials, out2);
    return hipGetLastError();
}

hipError_t launch_dd_update(long n, const double *e, double *hi, double *lo, hipStream_t s)
{
    hipLaunchKernelGGL(k_dd_update, grid_for(n), dim3(256), 0, s, n, e, hi, lo);
    return hipGetLastError();
}

hipError_t launch_build_coef(ToepCoef &c, hipStream_t s)
{
    long tot = (long)c.nq * 512 + c.n;
    hipLaunchKernelGGL(k_build_coef, grid_for(tot), dim3(256), 0, s, c.n, c.d64, c.d32, c.nq, c.fhi, c.flo);
    return hipGetLastError();
}

}  // namespace mgwr
