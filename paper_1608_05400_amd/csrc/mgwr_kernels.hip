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

#include <algorithm>
#include <cstdlib>
#include <type_traits>

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
    } else if constexpr (EPI == EPI_SCATTER_ADD) {
        double *o = e.out + (long)i * e.ldo + colour_point(e.dims, e.n, e.colour, p);
        *o = *o + acc;
    }
}

// Kernel parameters (passed by value).
struct KP {
    int M, P, K, off, ncoef;
    int tiles_m, tiles_n;
    int nsplit;                // K split factor (1: the product kernel applies the epilogue)
    const void *coef;          // double* or float* (F64/F32)
    const uint16_t *fhi, *flo; // fragment tables (BF16X3)
    const void *B;
    const uint16_t *Bhi, *Blo;
    long ldb;
    void *part;                // split partials [nsplit][M][P] (double for F64, float otherwise)
    EpiArgs ea;
};

// Work item b -> (row tile, column tile, split).  Row tiles in decreasing
// order (a causal product has the most work in its last rows, so the short
// tiles fill the tail of the launch); the splits of one tile are consecutive.
// With tiles_n a multiple of 8 the round-robin dispatch of blocks to the 8
// XCDs keeps each column strip of B on one XCD's L2.
struct Item {
    int tm, tn, s;
};
__device__ inline Item item_of(const KP &kp, int b)
{
    Item it;
    int t = b / kp.nsplit;
    it.s = b - t * kp.nsplit;
    it.tm = kp.tiles_m - 1 - t / kp.tiles_n;
    it.tn = t - (t / kp.tiles_n) * kp.tiles_n;
    return it;
}

// K range of the row tile [i0, i0 + BM): rows k with a nonzero coefficient
// t[off + i - k], in steps of BK from kbase; split s takes steps [ks0, ks1).
template <int BM, int BK>
__device__ inline void k_range(const KP &kp, int i0, int s, int &kbase, int &ks0, int &ks1)
{
    int kend = min(kp.K, i0 + BM + kp.off);
    int kbeg = max(0, kp.off + i0 - kp.ncoef + 1);
    kbeg = (kbeg / BK) * BK;
    int nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
    kbase = kbeg;
    ks0 = (int)((long)nk * s / kp.nsplit);
    ks1 = (int)((long)nk * (s + 1) / kp.nsplit);
}

// Result of element (i, p): the epilogue, or a partial sum when K is split.
template <int EPI, typename PT>
__device__ inline void emit(const KP &kp, int s, int i, int p, double acc)
{
    if (kp.nsplit > 1)
        ((PT *)kp.part)[((long)s * kp.M + i) * kp.P + p] = (PT)acc;
    else
        epi_apply<EPI>(kp.ea, i, p, acc);
}

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
// Wide FP64 / FP32 Toeplitz product.  Block of 4 waves arranged WGM x WGN,
// wave tile (16 FM) x (16 FN) of MFMA blocks; block tile BM x BN with
// BM = 16 FM WGM, BN = 16 FN WGN; K step 16; LDS double buffer for the B tile
// and the coefficient window (BM + BK - 1 values, from which every lane
// gathers its A element t[off + i - k]).
//   variant 0: 2 x 2 waves of 64 x 32   (block 128 x 64)
//   variant 1: 4 x 1 waves of 64 x 64   (block 256 x 64)
constexpr int WBK = 16, WBN = 64;
template <int V> struct WideCfg;
template <> struct WideCfg<0> { static constexpr int WGM = 2, WGN = 2, FM = 4, FN = 2; };
template <> struct WideCfg<1> { static constexpr int WGM = 4, WGN = 1, FM = 4, FN = 4; };
template <int V> constexpr int wide_bm() { return 16 * WideCfg<V>::FM * WideCfg<V>::WGM; }

template <int MODE, int EPI, int V>
__global__ __launch_bounds__(256) void k_toep_wide(KP kp)
{
    using T = Tr<MODE>;
    using S = typename T::S;
    using acc_t = typename T::acc_t;
    using C = WideCfg<V>;
    constexpr int BM = wide_bm<V>(), WIN = BM + WBK;
    static_assert(16 * C::FN * C::WGN == WBN, "block is 64 columns wide");
    __shared__ S Bs[2][WBK][WBN];
    __shared__ S Ws[2][WIN];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / C::WGN, wn = wid % C::WGN;
    const Item it = item_of(kp, blockIdx.x);
    const int i0 = it.tm * BM, p0 = it.tn * WBN;
    const S *coef = (const S *)kp.coef;
    const S *B = (const S *)kp.B;
    int kbase, ks0, ks1;
    k_range<BM, WBK>(kp, i0, it.s, kbase, ks0, ks1);
    const int nk = ks1 - ks0;
    const int kstart = kbase + ks0 * WBK;

    acc_t acc[C::FM][C::FN];
#pragma unroll
    for (int x = 0; x < C::FM; ++x)
#pragma unroll
        for (int y = 0; y < C::FN; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

    // staging: a wave loads one 64-column row of the B tile per instruction
    // (rows brow, brow + 4, brow + 8, brow + 12), fully coalesced for any ldb
    const int brow = tid >> 6, bcol = tid & 63;
    const bool colok = p0 + bcol < kp.P;
    S breg[4];
    S wreg0 = 0, wreg1 = 0;
    auto gload = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int k = k0 + brow + 4 * j;
            breg[j] = (k < kp.K && colok) ? B[(long)k * kp.ldb + p0 + bcol] : (S)0;
        }
        const int s0 = kp.off + i0 - k0 - (WBK - 1);
        if (tid < WIN) {
            int s = s0 + tid;
            wreg0 = (s >= 0 && s < kp.ncoef) ? coef[s] : (S)0;
        }
        if (tid + 256 < WIN) {
            int s = s0 + tid + 256;
            wreg1 = (s >= 0 && s < kp.ncoef) ? coef[s] : (S)0;
        }
    };
    auto sstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) Bs[buf][brow + 4 * j][bcol] = breg[j];
        if (tid < WIN) Ws[buf][tid] = wreg0;
        if (tid + 256 < WIN) Ws[buf][tid + 256] = wreg1;
    };

    if (nk > 0) {
        gload(kstart);
        sstore(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload(kstart + (kt + 1) * WBK);
#pragma unroll
        for (int ks = 0; ks < WBK / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            S a[C::FM], b[C::FN];
#pragma unroll
            for (int x = 0; x < C::FM; ++x)
                a[x] = Ws[buf][wm * 16 * C::FM + 16 * x + (lane & 15) - kr + WBK - 1];
#pragma unroll
            for (int y = 0; y < C::FN; ++y) b[y] = Bs[buf][kr][wn * 16 * C::FN + 16 * y + (lane & 15)];
#pragma unroll
            for (int x = 0; x < C::FM; ++x)
#pragma unroll
                for (int y = 0; y < C::FN; ++y) acc[x][y] = T::mma(a[x], b[y], acc[x][y]);
        }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < C::FM; ++x)
#pragma unroll
        for (int y = 0; y < C::FN; ++y) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int i = i0 + wm * 16 * C::FM + 16 * x + T::crow(lane, v);
                int p = p0 + wn * 16 * C::FN + 16 * y + (lane & 15);
                if (i < kp.M && p < kp.P) emit<EPI, S>(kp, it.s, i, p, (double)acc[x][y][v]);
            }
            // keep the read-modify-write epilogues from holding every load at once
            __builtin_amdgcn_sched_barrier(0);
        }
}

// ---------------------------------------------------------------------------
// Narrow Toeplitz product for levels with few columns (coarse grids): block
// tile 64 x 16; the four waves share the item's K range in chunks of 16 rows
// taken round-robin, and their partial tiles are summed in LDS in a fixed
// order.
constexpr int NBM = 64, NBN = 16, NCH = 16;

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void k_toep_narrow(KP kp)
{
    using T = Tr<MODE>;
    using S = typename T::S;
    using acc_t = typename T::acc_t;
    __shared__ S red[4][NBM * NBN];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const Item it = item_of(kp, blockIdx.x);
    const int i0 = it.tm * NBM, p0 = it.tn * NBN;
    const S *coef = (const S *)kp.coef;
    const S *B = (const S *)kp.B;
    int kbase, ks0, ks1;
    k_range<NBM, NCH>(kp, i0, it.s, kbase, ks0, ks1);

    acc_t acc[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) acc[x] = acc_t{0, 0, 0, 0};
    const int pc = p0 + (lane & 15);
    for (int c = ks0 + wid; c < ks1; c += 4) {
        const int k0 = kbase + c * NCH;
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
        if (i < kp.M && p < kp.P) emit<EPI, S>(kp, it.s, i, p, sum);
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 Toeplitz product.  Block tile 256 x 128, 4 waves in 2 x 2, wave
// tile 128 x 64 (8 x 4 blocks of 16 x 16, three v_mfma_f32_16x16x32_bf16 per
// block and K step of 32: lo*hi + hi*lo + hi*hi, each pass over all 32
// blocks so that an accumulator is reused only 32 MFMAs later).
//   * A (Toeplitz) fragments come straight from the fragment table (L2
//     resident) into registers.  The fragment of row block a at K step kt is
//     q = Q0 + a - 2 kt, so from one K step to the next six of the eight
//     stay in registers and only two new ones are loaded; they live in slot
//     (a - 2 kt) mod 8, a compile-time index once the K loop is unrolled by 4.
//   * B (k8-packed hi/lo, 16 KB per K step) goes global -> registers -> LDS
//     with three LDS buffers: the tile of step kt + 2 is loaded two steps
//     ahead (two register sets) and stored at the end of step kt, and the B
//     fragments of step kt + 1 are read from LDS while step kt's MFMAs run.
// B must be k8-packed with rows padded to a multiple of 256 and columns to a
// multiple of 128, padding zero.
constexpr int QBM = 256, QBN = 128, QBK = 32;

__device__ inline v8bf as_bf8(uint4 v) { return __builtin_bit_cast(v8bf, v); }

template <int EPI>
__global__ __launch_bounds__(256) void k_toep_bf16x3(KP kp)
{
    __shared__ uint4 Bs[3][2][4][QBN];   // [buffer][hi/lo][k/8][column]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const Item it = item_of(kp, blockIdx.x);
    const int i0 = it.tm * QBM, p0 = it.tn * QBN;
    int kbase, ks0, ks1;
    k_range<QBM, QBK>(kp, i0, it.s, kbase, ks0, ks1);
    const int nk = ks1 - ks0;
    const int kstart = kbase + ks0 * QBK;
    const int iw = i0 + wm * 128;
    const long Q0 = (kp.off + iw - kstart) / 16 + kQOff;   // fragment of row block 0 at K step 0

    v4f acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0, 0, 0, 0};

    const uint4 *fh = (const uint4 *)kp.fhi, *fl = (const uint4 *)kp.flo;
    const uint4 *bh = (const uint4 *)kp.Bhi, *bl = (const uint4 *)kp.Blo;
    const long ldb = kp.ldb;
    uint4 Ah[8], Al[8];          // Toeplitz fragment slots
    uint4 nh0, nl0, nh1, nl1;    // fragments of the next K step
    // two register sets for B tiles in flight: this thread's share is hi and
    // lo at rows k/8 = kr and kr + 2, column tc
    uint4 r00, r01, r02, r03, r10, r11, r12, r13;
    const int kr = tid >> 7, tc = tid & 127;
    // B fragments of this and of the next K step (two sets)
    v8bf fh0[4], fl0[4], fh1[4], fl1[4];
    const int fcol = wn * 64 + (lane & 15), frow = lane >> 4;

#define BF_GLOAD(R, KT)                                                                \
    {                                                                                  \
        const long rr = (kstart / 8) + 4L * (KT) + kr;                                 \
        R##0 = bh[rr * ldb + p0 + tc];                                                 \
        R##1 = bh[(rr + 2) * ldb + p0 + tc];                                           \
        R##2 = bl[rr * ldb + p0 + tc];                                                 \
        R##3 = bl[(rr + 2) * ldb + p0 + tc];                                           \
    }
#define BF_LSTORE(R, BUF)                                                              \
    {                                                                                  \
        Bs[BUF][0][kr][tc] = R##0;                                                     \
        Bs[BUF][0][kr + 2][tc] = R##1;                                                 \
        Bs[BUF][1][kr][tc] = R##2;                                                     \
        Bs[BUF][1][kr + 2][tc] = R##3;                                                 \
    }
#define BF_FREAD(FH, FL, BUF)                                                          \
    {                                                                                  \
        _Pragma("unroll") for (int b = 0; b < 4; ++b)                                  \
        {                                                                              \
            FH[b] = as_bf8(Bs[BUF][0][frow][fcol + 16 * b]);                           \
            FL[b] = as_bf8(Bs[BUF][1][frow][fcol + 16 * b]);                           \
        }                                                                              \
    }
#define BF_PASS(AX, BX, S)                                                             \
    _Pragma("unroll") for (int a = 0; a < 8; ++a)                                      \
        _Pragma("unroll") for (int b = 0; b < 4; ++b)                                  \
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(                       \
                as_bf8(AX[(a - 2 * (S)) & 7]), BX[b], acc[a][b], 0, 0, 0);
// one K step; S = KT mod 4 (compile time) selects the fragment slots and the
// register / fragment sets; the LDS buffer index is KT mod 3 (run time).  The
// loads and stores of a step are unconditional (indices clamped to the last
// step; a clamped store goes to the buffer no later step reads) so that the
// compiler's wait counts stay exact and the two-step prefetch survives.
#define BF_STEP(S, KT, RNEXT, RCUR, FHC, FLC, FHN, FLN)                                 \
    {                                                                                  \
        const int kt_ = (KT);                                                          \
        {                                                                              \
            const long q = Q0 - 2L * min(kt_ + 1, nk - 1);                             \
            nh0 = fh[q * 64 + lane];                                                   \
            nl0 = fl[q * 64 + lane];                                                   \
            nh1 = fh[(q + 1) * 64 + lane];                                             \
            nl1 = fl[(q + 1) * 64 + lane];                                             \
        }                                                                              \
        BF_GLOAD(RNEXT, min(kt_ + 3, nk - 1));                                         \
        BF_FREAD(FHN, FLN, (kt_ + 1) % 3);                                             \
        /* keep the loads above the MFMAs (the scheduler would sink them) */           \
        __builtin_amdgcn_sched_barrier(0);                                             \
        BF_PASS(Al, FHC, S)                                                            \
        BF_PASS(Ah, FLC, S)                                                            \
        BF_PASS(Ah, FHC, S)                                                            \
        __builtin_amdgcn_sched_barrier(0);                                             \
        BF_LSTORE(RCUR, (kt_ + 2) % 3);                                                \
        Ah[(0 - 2 * ((S) + 1)) & 7] = nh0;                                             \
        Al[(0 - 2 * ((S) + 1)) & 7] = nl0;                                             \
        Ah[(1 - 2 * ((S) + 1)) & 7] = nh1;                                             \
        Al[(1 - 2 * ((S) + 1)) & 7] = nl1;                                             \
        __syncthreads();                                                               \
    }

    if (nk > 0) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            Ah[a] = fh[(Q0 + a) * 64 + lane];
            Al[a] = fl[(Q0 + a) * 64 + lane];
        }
        BF_GLOAD(r0, 0);
        BF_GLOAD(r1, min(1, nk - 1));
        BF_LSTORE(r0, 0);
        BF_LSTORE(r1, 1);
        BF_GLOAD(r0, min(2, nk - 1));
    }
    __syncthreads();
    if (nk > 0) BF_FREAD(fh0, fl0, 0);
    // step kt: tile kt + 2 is in register set kt % 2, tile kt + 3 goes to the other
    int kt = 0;
    for (; kt + 4 <= nk; kt += 4) {
        BF_STEP(0, kt, r1, r0, fh0, fl0, fh1, fl1);
        BF_STEP(1, kt + 1, r0, r1, fh1, fl1, fh0, fl0);
        BF_STEP(2, kt + 2, r1, r0, fh0, fl0, fh1, fl1);
        BF_STEP(3, kt + 3, r0, r1, fh1, fl1, fh0, fl0);
    }
    if (kt < nk) {
        BF_STEP(0, kt, r1, r0, fh0, fl0, fh1, fl1);
        if (kt + 1 < nk) {
            BF_STEP(1, kt + 1, r0, r1, fh1, fl1, fh0, fl0);
            if (kt + 2 < nk) BF_STEP(2, kt + 2, r1, r0, fh0, fl0, fh1, fl1);
        }
    }
#undef BF_STEP
#undef BF_PASS
#undef BF_FREAD
#undef BF_LSTORE
#undef BF_GLOAD
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int i = iw + 16 * a + 4 * (lane >> 4) + v;
                int p = p0 + wn * 64 + 16 * b + (lane & 15);
                if (i < kp.M && p < kp.P) emit<EPI, float>(kp, it.s, i, p, (double)acc[a][b][v]);
            }
}

// Sum of the split partials in a fixed order, then the epilogue.
template <int EPI, typename PT>
__global__ void k_splitk_reduce(KP kp)
{
    const long MP = (long)kp.M * kp.P;
    const PT *part = (const PT *)kp.part;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < MP; e += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < kp.nsplit; ++s) acc += (double)part[s * MP + e];
        int i = (int)(e / kp.P), p = (int)(e - (long)i * kp.P);
        epi_apply<EPI>(kp.ea, i, p, acc);
    }
}

// ---------------------------------------------------------------------------
// Launch geometry.  A launch with few tiles (coarse levels) would leave most
// CUs idle while its last row tile walks the whole K range, so its K range
// is split over several blocks and a reduce kernel applies the epilogue.
struct Geo {
    int BM, BN, BK, tiles_m, tiles_n, nsplit, variant;
    size_t part_bytes;
};

// Wide-kernel variant per mode (0: 128 x 64 blocks, 1: 256 x 64 blocks,
// -1: by launch size); the environment variable MGWR_WIDE_VARIANT
// ("<fp64><fp32>", e.g. "10") fixes it for tuning runs.
static int wide_variant(int mode)
{
    static int v[2] = {-2, -2};
    if (v[0] == -2) {
        v[0] = -1; v[1] = -1;   // -1: choose by launch size
        const char *e = getenv("MGWR_WIDE_VARIANT");
        if (e && e[0] >= '0' && e[0] <= '1') v[0] = e[0] - '0';
        if (e && e[0] && e[1] >= '0' && e[1] <= '1') v[1] = e[1] - '0';
    }
    return v[mode == GM_F64 ? 0 : 1];
}

static Geo geometry(int mode, int M, int P, int K, int off, int ncoef, size_t part_cap)
{
    Geo g;
    g.variant = 0;
    if (mode == GM_BF16X3) { g.BM = QBM; g.BN = QBN; g.BK = QBK; }
    else if (P <= 32) { g.BM = NBM; g.BN = NBN; g.BK = NCH; }
    else {
        // 256-row blocks help launches that are too small to fill the chip
        // with 128-row blocks several times over
        const long t0 = (long)((M + wide_bm<0>() - 1) / wide_bm<0>()) * ((P + WBN - 1) / WBN);
        g.variant = wide_variant(mode);
        if (g.variant < 0) g.variant = (t0 < 4096) ? 1 : 0;
        g.BM = g.variant ? wide_bm<1>() : wide_bm<0>(); g.BN = WBN; g.BK = WBK;
    }
    g.tiles_m = (M + g.BM - 1) / g.BM;
    g.tiles_n = (P + g.BN - 1) / g.BN;
    const long T = (long)g.tiles_m * g.tiles_n;
    // K steps of the longest row tile
    int i0 = (g.tiles_m - 1) * g.BM;
    int kend = std::min(K, i0 + g.BM + off);
    int kbeg = std::max(0, off + i0 - ncoef + 1);
    int nk = (kend > kbeg) ? (kend - kbeg + g.BK - 1) / g.BK : 0;
    // target number of work items: the narrow kernel's items are short, so
    // it takes more of them; MGWR_SPLIT_TARGET overrides it for tuning runs
    static long tgt_env = -2;
    if (tgt_env == -2) {
        const char *e = getenv("MGWR_SPLIT_TARGET");
        tgt_env = e ? atol(e) : -1;
    }
    const long target = tgt_env > 0 ? tgt_env : (g.BM == NBM) ? 8192 : (mode == GM_BF16X3) ? 1024 : 2048;
    int ns = 1;
    if (T < target) {
        ns = (int)((target + T - 1) / T);
        ns = std::min(ns, 64);
        ns = std::min(ns, std::max(1, nk / 8));
    }
    const size_t esz = (mode == GM_F64) ? 8 : 4;
    while (ns > 1 && (size_t)ns * M * P * esz > part_cap) --ns;
    g.nsplit = ns;
    g.part_bytes = ns > 1 ? (size_t)ns * M * P * esz : 0;
    return g;
}

size_t splitk_bytes(int mode, int M, int P, int K, int off, int ncoef)
{
    return geometry(mode, M, P, K, off, ncoef, (size_t)-1).part_bytes;
}

static inline dim3 grid_for(long total, int threads = 256)
{
    long b = (total + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return dim3((unsigned)b);
}

template <int MODE, int EPI>
static hipError_t launch_mode_epi(const GemmArgs &a, KP &kp, hipStream_t s)
{
    Geo g = geometry(MODE, a.M, a.P, a.K, a.off, a.coef->n, a.part ? a.part_cap : 0);
    kp.tiles_m = g.tiles_m;
    kp.tiles_n = g.tiles_n;
    kp.nsplit = g.nsplit;
    kp.part = a.part;
    const unsigned blocks = (unsigned)((long)g.tiles_m * g.tiles_n * g.nsplit);
    if constexpr (MODE == GM_BF16X3) {
        hipLaunchKernelGGL((k_toep_bf16x3<EPI>), dim3(blocks), dim3(256), 0, s, kp);
    } else if (a.P <= 32) {
        hipLaunchKernelGGL((k_toep_narrow<MODE, EPI>), dim3(blocks), dim3(256), 0, s, kp);
    } else if (g.variant == 1) {
        hipLaunchKernelGGL((k_toep_wide<MODE, EPI, 1>), dim3(blocks), dim3(256), 0, s, kp);
    } else {
        hipLaunchKernelGGL((k_toep_wide<MODE, EPI, 0>), dim3(blocks), dim3(256), 0, s, kp);
    }
    if (g.nsplit > 1) {
        using PT = typename std::conditional<MODE == GM_F64, double, float>::type;
        hipLaunchKernelGGL((k_splitk_reduce<EPI, PT>), grid_for((long)a.M * a.P), dim3(256), 0, s, kp);
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(const GemmArgs &a, KP &kp, hipStream_t s)
{
    switch (a.epi) {
    case EPI_STORE: return launch_mode_epi<MODE, EPI_STORE>(a, kp, s);
    case EPI_SCATTER: return launch_mode_epi<MODE, EPI_SCATTER>(a, kp, s);
    case EPI_SCATTER_ADD: return launch_mode_epi<MODE, EPI_SCATTER_ADD>(a, kp, s);
    case EPI_SUB: return launch_mode_epi<MODE, EPI_SUB>(a, kp, s);
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
__global__ void k_rhs_panel(int dims, int n, int colour, int M, int Pc, const double *F, double *U,
                            const double *cd, const double *g, double ih2, double lam0, S *panel,
                            long ldp)
{
    long P = (dims == 1) ? n : (long)n * n;
    long total = (long)M * Pc;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int k = (int)(e / Pc), j = (int)(e - (long)k * Pc);
        int pt = colour_point(dims, n, colour, j);
        double *Uk = U + (long)k * P;
        double b = F[(long)k * P + pt] + nbr_sum(Uk, dims, n, pt) * ih2;
        if (g) b += cd[k] * g[pt];
        panel[(long)k * ldp + j] = (S)b;
        if (lam0 != 0.0) Uk[pt] = lam0 * b;
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
                                   const double *F, double *U, const double *cd, const double *g,
                                   double ih2, double lam0, uint16_t *hi, uint16_t *lo, long ldp)
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
                double *Uk = U + (long)k * P;
                b = F[(long)k * P + pt] + nbr_sum(Uk, dims, n, pt) * ih2;
                if (g) b += cd[k] * g[pt];
                if (lam0 != 0.0) Uk[pt] = lam0 * b;
            }
            b8[q] = (float)b;
        }
        store_split8(b8, hi, lo, e);
    }
}

// Residual (Section 2, eq. discrete_model_IVP_1; Section 6) from the Toeplitz
// product already stored in out: out = (f + c d g - diag u - A_h u) - out.
// With lo != nullptr the iterate is the double-double hi + lo and A_h is
// applied with error-free transformations.
__global__ void k_resid_post(int dims, int n, int M, const double *F, const double *U, const double *lo,
                             const double *cd, const double *g, double ih2, double diag, double *out)
{
    long P = (dims == 1) ? n : (long)n * n;
    long total = (long)M * P;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int k = (int)(e / P), p = (int)(e - (long)k * P);
        const double *Uk = U + (long)k * P;
        double rhs = F[e];
        if (g) rhs += cd[k] * g[p];
        if (diag != 0.0) rhs -= diag * Uk[p];
        double r;
        if (lo) {
            double shi, slo;
            stencil_dd(Uk, lo + (long)k * P, dims, n, p, shi, slo);
            r = (rhs - shi * ih2) - slo * ih2;
        } else {
            double st = (dims == 1 ? 2.0 : 4.0) * Uk[p] - nbr_sum(Uk, dims, n, p);
            r = rhs - st * ih2;
        }
        out[e] = r - out[e];
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

__global__ void k_scaled_fill(long M, long P, const double *cd, const double *g, double *u)
{
    long total = M * P;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        u[e] = g ? cd[e / P] * g[e % P] : 0.0;
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
hipError_t launch_rhs_panel(int fmt, int dims, int n, int colour, int M, int Mpad, const double *F,
                            double *U, const double *cd, const double *g, double ih2, double lam0,
                            void *panel, void *panel_lo, long ldp, hipStream_t s)
{
    int Pc = colour_count(dims, n, colour);
    if (fmt == 2) {
        long total = (long)(Mpad / 8) * ldp;
        hipLaunchKernelGGL(k_rhs_panel_packed, grid_for(total), dim3(256), 0, s, dims, n, colour, M, Mpad,
                           Pc, F, U, cd, g, ih2, lam0, (uint16_t *)panel, (uint16_t *)panel_lo, ldp);
    } else if (fmt == 0) {
        hipLaunchKernelGGL(k_rhs_panel<double>, grid_for((long)M * Pc), dim3(256), 0, s, dims, n, colour,
                           M, Pc, F, U, cd, g, ih2, lam0, (double *)panel, ldp);
    } else {
        hipLaunchKernelGGL(k_rhs_panel<float>, grid_for((long)M * Pc), dim3(256), 0, s, dims, n, colour,
                           M, Pc, F, U, cd, g, ih2, lam0, (float *)panel, ldp);
    }
    return hipGetLastError();
}

hipError_t launch_resid_post(int dims, int n, int M, const double *F, const double *U, const double *lo,
                             const double *cd, const double *g, double ih2, double diag, double *out,
                             hipStream_t s)
{
    long total = (long)M * ((dims == 1) ? n : (long)n * n);
    hipLaunchKernelGGL(k_resid_post, grid_for(total), dim3(256), 0, s, dims, n, M, F, U, lo, cd, g, ih2, diag,
                       out);
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

hipError_t launch_scaled_fill(long M, long P, const double *cd, const double *g, double *u, hipStream_t s)
{
    hipLaunchKernelGGL(k_scaled_fill, grid_for(M * P), dim3(256), 0, s, M, P, cd, g, u);
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
