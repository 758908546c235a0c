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
#include <cmath>
#include <cstdlib>
#include <map>
#include <type_traits>

namespace mgwr {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Global-memory views of pointers that reach a kernel inside an argument
// struct (by value or from a device array): without them the compiler cannot
// tell global from LDS or scratch and issues flat accesses, whose completion
// the wait counters of both memory paths must cover.
#define GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ inline const GLOBAL T *gview(const void *p) { return (const GLOBAL T *)p; }
template <typename T> __device__ inline GLOBAL T *gview_rw(void *p) { return (GLOBAL T *)p; }

// ---------------------------------------------------------------------------
// BF16 helpers: round-to-nearest-even of a finite float, and back.
__device__ inline uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

#define RET_IF(e)                          \
    do {                                   \
        hipError_t e_ = (e);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

// ---------------------------------------------------------------------------
// Stencils of the negative Laplacian (Section 2: 3-point; Section 6: 5-point)
// with zero Dirichlet values, on one time row U of a level with n points/dim.
// The neighbours are loaded at clamped indices and the ones outside the grid
// replaced by zero, so that no load sits behind a branch.
// p is the natural index of the point; the row is stored in the order
// `split` (lay_pos).
template <typename Ptr>
__device__ inline void nbr_vals_xy(Ptr U, int n, int x, int y, double (&v)[4], int split)
{
    v[0] = (double)U[lay_pos_xy(n, split, x > 0 ? x - 1 : x, y)];
    v[1] = (double)U[lay_pos_xy(n, split, x < n - 1 ? x + 1 : x, y)];
    v[2] = (double)U[lay_pos_xy(n, split, x, y > 0 ? y - 1 : y)];
    v[3] = (double)U[lay_pos_xy(n, split, x, y < n - 1 ? y + 1 : y)];
    if (x == 0) v[0] = 0.0;
    if (x == n - 1) v[1] = 0.0;
    if (y == 0) v[2] = 0.0;
    if (y == n - 1) v[3] = 0.0;
}
template <typename Ptr>
__device__ inline void nbr_vals(Ptr U, int dims, int n, int p, double (&v)[4], int split = 0)
{
    if (dims == 2) {
        const int y = p / n;
        nbr_vals_xy(U, n, p - y * n, y, v, split);
        return;
    }
    // a 1D row is an n x 1 grid: its y-neighbours are outside
    v[0] = (double)U[lay_pos(1, n, split, p > 0 ? p - 1 : p)];
    v[1] = (double)U[lay_pos(1, n, split, p < n - 1 ? p + 1 : p)];
    v[2] = v[3] = 0.0;
    if (p == 0) v[0] = 0.0;
    if (p == n - 1) v[1] = 0.0;
}

template <typename Ptr>
__device__ inline double nbr_sum_xy(Ptr U, int n, int x, int y, int split)
{
    double v[4];
    nbr_vals_xy(U, n, x, y, v, split);
    return ((v[0] + v[1]) + v[2]) + v[3];
}
template <typename Ptr>
__device__ inline double nbr_sum(Ptr U, int dims, int n, int p, int split = 0)
{
    double v[4];
    nbr_vals(U, dims, n, p, v, split);
    return ((v[0] + v[1]) + v[2]) + v[3];
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
__device__ inline void stencil_dd_vals(double hc, double lc, const double (&h)[4], const double (&l)[4], double d,
                                       double &shi, double &slo)
{
    double s = d * hc, e, acc = 0.0;
    double lo = d * lc;
#pragma unroll
    for (int k = 0; k < 4; ++k) {   // a zero neighbour leaves s exact and adds nothing
        two_sum(s, -h[k], s, e);
        acc += e;
        lo -= l[k];
    }
    shi = s;
    slo = acc + lo;
}
template <typename Ptr>
__device__ inline void stencil_dd(Ptr H, Ptr Lo, int dims, int n, int p, double &shi, double &slo, int split = 0)
{
    double h[4], l[4];
    int sp;
    if (dims == 2) {
        const int y = p / n, x = p - y * n;
        nbr_vals_xy(H, n, x, y, h, split);
        nbr_vals_xy(Lo, n, x, y, l, split);
        sp = lay_pos_xy(n, split, x, y);
    } else {
        nbr_vals(H, 1, n, p, h, split);
        nbr_vals(Lo, 1, n, p, l, split);
        sp = lay_pos(1, n, split, p);
    }
    stencil_dd_vals(H[sp], Lo[sp], h, l, dims == 1 ? 2.0 : 4.0, shi, slo);
}
// The same at the 2D point (x, y) stored at sp.
template <typename Ptr>
__device__ inline void stencil_dd_xy(Ptr H, Ptr Lo, int n, int x, int y, int sp, double &shi, double &slo, int split)
{
    double h[4], l[4];
    nbr_vals_xy(H, n, x, y, h, split);
    nbr_vals_xy(Lo, n, x, y, l, split);
    stencil_dd_vals(H[sp], Lo[sp], h, l, 4.0, shi, slo);
}

// Right-hand side of the smoother (Section 3, eq. red-black; Section 6, eq.
// red-black_2d) at time row i and the j-th point of a colour, on a level
// stored split by colour: f + (neighbour sum) / h^2 + c d_i g (EpiArgs::rhs).
// In 1D the neighbours of colour 0's point j are the other colour's points
// j and j + 1, those of colour 1's point j the other's j - 1 and j (each
// inside the grid); loads at clamped indices.
__device__ inline double rhs_val(const EpiArgs &e, int i, int j)
{
    const long k = (long)i * e.ldu;
    const GLOBAL double *Uk = gview<double>(e.U) + k;
    double b = gview<double>(e.F)[k + j];
    double ns;
    if (e.dims == 1) {
        const int o = e.colour == 0 ? e.n / 2 : 0;            // the other colour's first point
        const int po = e.colour == 0 ? (e.n + 1) / 2 : e.n / 2;   // and its count (0 when n = 1)
        const int jl = e.colour == 0 ? j : j - 1, jr = e.colour == 0 ? j + 1 : j;
        // loads clamped into the level's row (the other colour may be empty)
        double vl = Uk[min(max(o + jl, 0), e.n - 1)], vr = Uk[min(max(o + jr, 0), e.n - 1)];
        if (jl < 0 || jl >= po) vl = 0.0;
        if (jr < 0 || jr >= po) vr = 0.0;
        ns = vl + vr;
    } else {
        int x, y;
        colour_xy(e.n, e.colour, j, x, y);
        ns = nbr_sum_xy(Uk, e.n, x, y, 1);
    }
    b += ns * e.ih2;
    if (e.g) b += gview<double>(e.cd)[i] * gview<double>(e.g)[colour_point(e.dims, e.n, e.colour, j)];
    return b;
}

// ---------------------------------------------------------------------------
// Epilogue of the Toeplitz products, element (i, p) with product value acc,
// in two parts so that a thread can issue the loads of all its elements
// before any store (a store may alias a later load, so interleaved
// read-modify-writes would wait for every load in turn): epi_pre reads what
// the element needs, epi_put combines it with acc and stores.
template <int EPI>
__device__ inline double epi_pre(const EpiArgs &e, int i, int p)
{
    const GLOBAL double *out = gview<double>(e.out);
    if constexpr (EPI == EPI_SUB || EPI == EPI_ADD) {
        return out[(long)i * e.ldo + p];
    } else if constexpr (EPI == EPI_STORE_DIAG) {
        return e.diag * gview<double>(e.b)[(long)i * e.ldb_diag + p];
    } else if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_DD || EPI == EPI_RESID_C || EPI == EPI_RESID_R) {
        // the stencil part of the residual (as OpPost), fused; no load
        // behind a divergent branch (g and cd are read only when there is an
        // initial condition, a launch-wide choice; diag = 0 subtracts an
        // exact zero).  nat: the natural point, sp: its storage index (F, U
        // and lo in the order lay_in; column p is the colour's p-th point for
        // the one-colour residuals, else storage index p)
        int nat, sp;
        if constexpr (EPI == EPI_RESID_C || EPI == EPI_RESID_R) {
            nat = colour_point(e.dims, e.n, e.colour, p);
            sp = lay_cpos(e.dims, e.n, e.lay_in, e.colour, p);
        } else {
            nat = lay_nat(e.dims, e.n, e.lay_in, p);
            sp = p;
        }
        const long k = (long)i * e.ldu;
        const GLOBAL double *Uk = gview<double>(e.U) + k;
        double rhs = gview<double>(e.F)[k + sp];
        if (e.g) rhs += gview<double>(e.cd)[i] * gview<double>(e.g)[nat];
        rhs -= e.diag * Uk[sp];
        if constexpr (EPI == EPI_RESID_DD) {
            double shi, slo;
            stencil_dd(Uk, gview<double>(e.lo) + k, e.dims, e.n, nat, shi, slo, e.lay_in);
            return (rhs - shi * e.ih2) - slo * e.ih2;
        } else {
            double st = (e.dims == 1 ? 2.0 : 4.0) * Uk[sp] - nbr_sum(Uk, e.dims, e.n, nat, e.lay_in);
            return rhs - st * e.ih2;
        }
    } else {
        return 0.0;
    }
}

template <int EPI>
__device__ inline void epi_put(const EpiArgs &e, int i, int p, double pre, double acc)
{
    GLOBAL double *out = gview_rw<double>(e.out);
    if constexpr (EPI == EPI_STORE) {
        out[(long)i * e.ldo + p] = acc;
    } else if constexpr (EPI == EPI_SUB) {
        out[(long)i * e.ldo + p] = pre - acc;
    } else if constexpr (EPI == EPI_ADD) {
        out[(long)i * e.ldo + p] = pre + acc;
    } else if constexpr (EPI == EPI_SCATTER) {
        out[(long)i * e.ldo + colour_point(e.dims, e.n, e.colour, p)] = acc;
    } else if constexpr (EPI == EPI_STORE_DIAG) {
        out[(long)i * e.ldo + p] = pre + acc;
    } else if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_DD) {
        const int q = (e.lay_out == e.lay_in) ? p
                      : lay_pos(e.dims, e.n, e.lay_out, lay_nat(e.dims, e.n, e.lay_in, p));
        out[(long)i * e.ldo + q] = pre - acc;
    } else if constexpr (EPI == EPI_RESID_C) {
        out[(long)i * e.ldo + lay_cpos(e.dims, e.n, e.lay_out, e.colour, p)] = pre - acc;
    } else if constexpr (EPI == EPI_RESID_R) {
        // colour 0's p-th fine point is coarse point p (natural)
        out[(long)i * e.ldo + lay_pos(1, (e.n - 1) / 2, e.lay_out, p)] = 0.25 * (2.0 * (pre - acc));
    }
}

// Residual epilogue values (as epi_pre) of points p and p + S of row i on a
// 1D level (S = 1: adjacent points; S = 2: adjacent points of one colour),
// the second only meaningful when p + S < n: the neighbour values the two
// share are loaded once, at clamped indices.
template <bool DD, int S>
__device__ inline void resid_pre_pair_1d(const EpiArgs &e, int i, int p, double &r0, double &r1)
{
    const int n = e.n;
    const long k = (long)i * e.ldu;
    const int pl = p > 0 ? p - 1 : p, p1 = min(p + S, n - 1), p2 = min(p + S + 1, n - 1), pm = min(p + 1, n - 1);
    const GLOBAL double *Uk = gview<double>(e.U) + k, *Fk = gview<double>(e.F) + k;
    const GLOBAL double *g = gview<double>(e.g);
    double uL = Uk[pl], u0 = Uk[p], u1 = Uk[p1], uR = Uk[p2];
    const double uM = (S == 2) ? Uk[pm] : u1;   // right of p (and left of p + 2)
    const double f0 = Fk[p], f1 = Fk[p1];
    double g0 = 0.0, g1 = 0.0, cdv = 0.0;
    if (e.g) {   // a launch-wide choice
        g0 = g[p];
        g1 = g[p1];
        cdv = gview<double>(e.cd)[i];
    }
    double lL = 0.0, l0 = 0.0, l1 = 0.0, lR = 0.0, lM = 0.0;
    if constexpr (DD) {
        const GLOBAL double *Lk = gview<double>(e.lo) + k;
        lL = Lk[pl]; l0 = Lk[p]; l1 = Lk[p1]; lR = Lk[p2];
        lM = (S == 2) ? Lk[pm] : l1;
    }
    if (p == 0) uL = lL = 0.0;
    // neighbours: right of p, left of p + S, right of p + S (zero outside)
    const double ur0 = (p + 1 < n) ? uM : 0.0, ul1 = (S == 1) ? u0 : uM, ur1 = (p + S + 1 < n) ? uR : 0.0;
    const double lr0 = (p + 1 < n) ? lM : 0.0, ll1 = (S == 1) ? l0 : lM, lr1 = (p + S + 1 < n) ? lR : 0.0;
    double rhs0 = f0, rhs1 = f1;
    if (e.g) {
        rhs0 += cdv * g0;
        rhs1 += cdv * g1;
    }
    rhs0 -= e.diag * u0;
    rhs1 -= e.diag * u1;
    if constexpr (DD) {
        // stencil_dd of both points
        double s0 = 2.0 * u0, s1 = 2.0 * u1, e0, e1, a0 = 0.0, a1 = 0.0;
        double lo0 = 2.0 * l0, lo1 = 2.0 * l1;
        two_sum(s0, -uL, s0, e0); a0 += e0; lo0 -= lL;
        two_sum(s0, -ur0, s0, e0); a0 += e0; lo0 -= lr0;
        two_sum(s1, -ul1, s1, e1); a1 += e1; lo1 -= ll1;
        two_sum(s1, -ur1, s1, e1); a1 += e1; lo1 -= lr1;
        r0 = (rhs0 - s0 * e.ih2) - (a0 + lo0) * e.ih2;
        r1 = (rhs1 - s1 * e.ih2) - (a1 + lo1) * e.ih2;
    } else {
        r0 = rhs0 - (2.0 * u0 - (uL + ur0)) * e.ih2;
        r1 = rhs1 - (2.0 * u1 - (ul1 + ur1)) * e.ih2;
    }
}

// Rows of a thread's outputs whose epilogue loads are issued together (of
// n): the residual's stencil reads several values per element, so one row
// (two elements) at a time keeps them in registers (measured 4 % faster than
// two rows, 20 % faster than four).
template <int EPI> __host__ __device__ constexpr int epi_rows(int n)
{
    return (EPI == EPI_RESID || EPI == EPI_RESID_DD || EPI == EPI_RESID_C || EPI == EPI_RESID_R) ? 1 : n;
}

template <int EPI>
__device__ inline void epi_apply(const EpiArgs &e, int i, int p, double acc)
{
    epi_put<EPI>(e, i, p, epi_pre<EPI>(e, i, p), acc);
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

// One launch of a product kernel over the products of several problems:
// block b runs work item items[b].y of problem items[b].x; the host sorts the
// table by the K extent of the items, longest first, so that the short items
// of every problem fill the tail of the launch.
struct KGrp {
    KP one;                    // the product when n == 1 (block b = item b)
    const KP *many;            // n > 1: device array of n products
    const int2 *items;         // n > 1: (product, work item) of every block
    int n;
};
__device__ inline void kgrp_select(const KGrp &g, KP &kp, int &b)
{
    if (g.n == 1) {
        kp = g.one;
        b = blockIdx.x;
        return;
    }
    const int2 it = g.items[blockIdx.x];
    const int p = __builtin_amdgcn_readfirstlane(it.x);
    b = __builtin_amdgcn_readfirstlane(it.y);
    kp = g.many[p];
}

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

// Pieces of the epilogues for the product kernels: the output column of
// product column p, whether the epilogue reads the old value, and the new value.
template <int EPI> __device__ constexpr bool epi_reads()
{
    return EPI == EPI_SUB || EPI == EPI_ADD;
}
template <int EPI> __device__ inline long epi_col(const EpiArgs &e, int p)
{
    if constexpr (EPI == EPI_SCATTER) return colour_point(e.dims, e.n, e.colour, p);
    else return p;
}
template <int EPI> __device__ inline double epi_combine(double prev, double acc)
{
    if constexpr (EPI == EPI_SUB) return prev - acc;
    else if constexpr (EPI == EPI_ADD) return prev + acc;
    else return acc;
}

// Result of element (i, p): the epilogue, or a partial sum when K is split.
template <int EPI, typename PT>
__device__ inline void emit(const KP &kp, int s, int i, int p, double acc)
{
    if (kp.nsplit > 1)
        gview_rw<PT>(kp.part)[((long)s * kp.M + i) * kp.P + p] = (PT)acc;
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
__global__ __launch_bounds__(256) void k_toep_wide(KGrp grp)
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
    KP kp;
    int blk;
    kgrp_select(grp, kp, blk);
    const Item it = item_of(kp, blk);
    const int i0 = it.tm * BM, p0 = it.tn * WBN;
    const GLOBAL S *coef = gview<S>(kp.coef);
    const GLOBAL S *B = gview<S>(kp.B);
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
    const int pl = p0 + wn * 16 * C::FN + (lane & 15);
    if (kp.nsplit > 1) {
#pragma unroll
        for (int x = 0; x < C::FM; ++x)
#pragma unroll
            for (int y = 0; y < C::FN; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i = i0 + wm * 16 * C::FM + 16 * x + T::crow(lane, v);
                    int p = pl + 16 * y;
                    if (i < kp.M && p < kp.P) emit<EPI, S>(kp, it.s, i, p, (double)acc[x][y][v]);
                }
        return;
    }
    // one row block at a time: all old values of the block are loaded before
    // any store (a load cannot move above a store to the same array, so an
    // interleaved read-modify-write would wait for every load in turn)
    GLOBAL double *out = gview_rw<double>(kp.ea.out);
    long col[C::FN];
    bool cok[C::FN];
#pragma unroll
    for (int y = 0; y < C::FN; ++y) {
        cok[y] = pl + 16 * y < kp.P;
        col[y] = cok[y] ? epi_col<EPI>(kp.ea, pl + 16 * y) : 0;
    }
#pragma unroll
    for (int x = 0; x < C::FM; ++x) {
        double prev[C::FN][4];
#pragma unroll
        for (int y = 0; y < C::FN; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 16 * C::FM + 16 * x + T::crow(lane, v);
                prev[y][v] = 0.0;
                if constexpr (epi_reads<EPI>())
                    if (cok[y] && i < kp.M) prev[y][v] = out[(long)i * kp.ea.ldo + col[y]];
            }
#pragma unroll
        for (int y = 0; y < C::FN; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 16 * C::FM + 16 * x + T::crow(lane, v);
                if (cok[y] && i < kp.M)
                    out[(long)i * kp.ea.ldo + col[y]] = epi_combine<EPI>(prev[y][v], (double)acc[x][y][v]);
            }
    }
}

// ---------------------------------------------------------------------------
// Narrow Toeplitz product for levels with few columns (coarse grids): block
// tile 64 x 16; the four waves share the item's K range in chunks of 16 rows
// taken round-robin, and their partial tiles are summed in LDS in a fixed
// order.
constexpr int NBM = 64, NBN = 16, NCH = 16;

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void k_toep_narrow(KGrp grp)
{
    using T = Tr<MODE>;
    using S = typename T::S;
    using acc_t = typename T::acc_t;
    __shared__ S red[4][NBM * NBN];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    KP kp;
    int blk;
    kgrp_select(grp, kp, blk);
    const Item it = item_of(kp, blk);
    const int i0 = it.tm * NBM, p0 = it.tn * NBN;
    const GLOBAL S *coef = gview<S>(kp.coef);
    const GLOBAL S *B = gview<S>(kp.B);
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

__device__ inline v8bf as_bf8(u32x4 v) { return __builtin_bit_cast(v8bf, v); }

template <int EPI>
__global__ __launch_bounds__(256) void k_toep_bf16x3(KGrp grp)
{
    __shared__ u32x4 Bs[3][2][4][QBN];   // [buffer][hi/lo][k/8][column]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    KP kp;
    int blk;
    kgrp_select(grp, kp, blk);
    const Item it = item_of(kp, blk);
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

    const GLOBAL u32x4 *fh = gview<u32x4>(kp.fhi), *fl = gview<u32x4>(kp.flo);
    const GLOBAL u32x4 *bh = gview<u32x4>(kp.Bhi), *bl = gview<u32x4>(kp.Blo);
    const long ldb = kp.ldb;
    u32x4 Ah[8], Al[8];          // Toeplitz fragment slots
    u32x4 nh0, nl0, nh1, nl1;    // fragments of the next K step
    // two register sets for B tiles in flight: this thread's share is hi and
    // lo at rows k/8 = kr and kr + 2, column tc
    u32x4 r00, r01, r02, r03, r10, r11, r12, r13;
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
    const int pl = p0 + wn * 64 + (lane & 15);
    if (kp.nsplit > 1) {
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int i = iw + 16 * a + 4 * (lane >> 4) + v;
                    int p = pl + 16 * b;
                    if (i < kp.M && p < kp.P) emit<EPI, float>(kp, it.s, i, p, (double)acc[a][b][v]);
                }
        return;
    }
    GLOBAL double *out = gview_rw<double>(kp.ea.out);
    const long ldo = kp.ea.ldo;
    long col[4];
    bool cok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        cok[b] = pl + 16 * b < kp.P;
        col[b] = cok[b] ? epi_col<EPI>(kp.ea, pl + 16 * b) : 0;
    }
    // A wave whose 128 x 64 tile lies inside the product (every tile but the
    // last column strip's and a ragged M's) writes it without per-element
    // predicates, its loads of the old values (read-modify-write epilogues)
    // one row block ahead of the stores: predicated accesses split the
    // epilogue into branches whose stores the compiler waits for one by one,
    // and at one wave per SIMD that idles the matrix cores.
    const bool inner = __builtin_amdgcn_readfirstlane((int)(iw + 128 <= kp.M && p0 + wn * 64 + 64 <= kp.P));
    if (inner) {
        GLOBAL double *ob = out + (long)(iw + 4 * (lane >> 4)) * ldo;
        double prev[2][4][4];
        auto load_rows = [&](int a, double (&pv)[4][4]) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) pv[b][v] = ob[(long)(16 * a + v) * ldo + col[b]];
        };
        if constexpr (epi_reads<EPI>()) load_rows(0, prev[0]);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if constexpr (epi_reads<EPI>())
                if (a + 1 < 8) load_rows(a + 1, prev[(a + 1) & 1]);
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double pv = epi_reads<EPI>() ? prev[a & 1][b][v] : 0.0;
                    ob[(long)(16 * a + v) * ldo + col[b]] = epi_combine<EPI>(pv, (double)acc[a][b][v]);
                }
        }
        return;
    }
    // edge tiles: one row block at a time, its loads before its stores
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        double prev[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = iw + 16 * a + 4 * (lane >> 4) + v;
                prev[b][v] = 0.0;
                if constexpr (epi_reads<EPI>())
                    if (cok[b] && i < kp.M) prev[b][v] = out[(long)i * ldo + col[b]];
            }
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = iw + 16 * a + 4 * (lane >> 4) + v;
                if (cok[b] && i < kp.M)
                    out[(long)i * ldo + col[b]] = epi_combine<EPI>(prev[b][v], (double)acc[a][b][v]);
            }
    }
}

// ---------------------------------------------------------------------------
// Grouped launches of the bandwidth kernels: block b of the launch runs block
// b - start[p] of argument set p, where start[] is the prefix sum of the
// blocks each set asked for; a set of one is passed by value.
template <class A> struct Grp {
    A one;
    const A *many;
    const int *start;   // n + 1 entries
    int n;
};

// Number of i in [1, n) with start[i] <= b, i.e. the set that owns block b
// (each wave counts on its own: no LDS, no barrier).
__device__ inline int grp_find(const int *start, int n, int b)
{
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    for (int base = 1; base < n; base += 64) {
        const int i = base + lane;
        const bool le = (i < n) && (start[i] <= b);
        cnt += __popcll(__ballot(le));
    }
    return cnt;
}

template <class A>
__device__ inline void grp_select(const Grp<A> &g, A &a, long &lb, long &nb)
{
    if (g.n == 1) {
        a = g.one;
        lb = blockIdx.x;
        nb = gridDim.x;
        return;
    }
    const int p = __builtin_amdgcn_readfirstlane(grp_find(g.start, g.n, blockIdx.x));
    a = g.many[p];
    const int s0 = g.start[p], s1 = g.start[p + 1];
    lb = (long)blockIdx.x - s0;
    nb = s1 - s0;
}

constexpr int kThreads = 256;
// Whether a launch argument set has a `dims` member (the level's dimension).
template <class A, class = void> struct HasDims : std::false_type {};
template <class A> struct HasDims<A, std::void_t<decltype(std::declval<A>().dims)>> : std::true_type {};
#define GRID_STRIDE(e, total) \
    for (long e = lb * kThreads + threadIdx.x; e < (total); e += nb * kThreads)

// The same walk over the (row, column) pairs (k, s) of rows of P elements,
// without a 64-bit division per element: the stride is split once into whole
// rows and a remainder.
struct KsWalk {
    long k, dk;
    int s, ds, P;
    __device__ KsWalk(long lb, long nb, int P_) : P(P_)
    {
        if (P <= 0) {   // empty rows: no pair (k never below a row count)
            k = 0x7fffffffffffffffL;
            dk = 0;
            s = ds = 0;
            return;
        }
        const long e = lb * kThreads + threadIdx.x, st = nb * kThreads;
        k = e / P;
        s = (int)(e - k * P);
        dk = st / P;
        ds = (int)(st - dk * P);
    }
    __device__ void next()
    {
        s += ds;
        k += dk;
        if (s >= P) {
            s -= P;
            ++k;
        }
    }
};

template <class Op>
__global__ __launch_bounds__(kThreads) void k_group(Grp<typename Op::A> g)
{
    typename Op::A a;
    long lb, nb;
    grp_select(g, a, lb, nb);
    // Blocks go to the 8 XCDs in turn.  On a 2D level, when the set's blocks
    // fill whole rounds, they are renumbered so that each XCD runs one
    // contiguous eighth of them: a 5-point stencil's neighbour rows are then
    // read through the same L2 (2D N = 1023 step 976 -> 939 ms, N = 511
    // 529 -> 521 ms; the same on the 1D workloads measured 2 % slower).
    if constexpr (HasDims<typename Op::A>::value)
        if (a.dims == 2 && (nb & 7) == 0 && ((blockIdx.x - lb) & 7) == 0) lb = (lb & 7) * (nb >> 3) + (lb >> 3);
    Op::run(a, lb, nb);
}

// Sum of the split partials in a fixed order, then the epilogue.
template <int EPI, typename PT> struct OpReduce {
    using A = KP;
    __device__ static void run(const KP &kp, long lb, long nb)
    {
        const long MP = (long)kp.M * kp.P;
        const GLOBAL PT *part = gview<PT>(kp.part);
        GRID_STRIDE(e, MP) {
            double acc = 0.0;
            for (int s = 0; s < kp.nsplit; ++s) acc += (double)part[s * MP + e];
            int i = (int)(e / kp.P), p = (int)(e - (long)i * kp.P);
            epi_apply<EPI>(kp.ea, i, p, acc);
        }
    }
};

// ---------------------------------------------------------------------------
// Launch geometry of the products.  kind: 0 narrow (64 x 16 blocks), 1 wide
// 128 x 64, 2 wide 256 x 64, 3 split-BF16 256 x 128.
struct Geo {
    int kind, BM, BN, BK, tiles_m, tiles_n, nsplit;
    size_t part_bytes;
};

static int tile_steps(int K, int off, int ncoef, int BM, int BK, int tm)
{
    const int i0 = tm * BM;
    const int kend = std::min(K, i0 + BM + off);
    int kbeg = std::max(0, off + i0 - ncoef + 1);
    kbeg = (kbeg / BK) * BK;
    return (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
}

static Geo tiles(int mode, int M, int P, const TileKnobs &kn)
{
    Geo g{};
    if (mode == GM_BF16X3) { g.kind = 3; g.BM = QBM; g.BN = QBN; g.BK = QBK; }
    else if (P <= 32) { g.kind = 0; g.BM = NBM; g.BN = NBN; g.BK = NCH; }
    else {
        // 256-row blocks help launches too small to fill the chip several
        // times over with 128-row blocks
        const long t0 = (long)((M + wide_bm<0>() - 1) / wide_bm<0>()) * ((P + WBN - 1) / WBN);
        int v = kn.variant;
        if (v < 0) v = (t0 < 4096) ? 1 : 0;
        g.kind = 1 + v; g.BM = v ? wide_bm<1>() : wide_bm<0>(); g.BN = WBN; g.BK = WBK;
    }
    g.tiles_m = (M + g.BM - 1) / g.BM;
    g.tiles_n = (P + g.BN - 1) / g.BN;
    g.nsplit = 1;
    g.part_bytes = 0;
    return g;
}

static int split_cap(int mode, int M, int P, int ns, size_t part_cap)
{
    const size_t esz = (mode == GM_F64) ? 8 : 4;
    while (ns > 1 && (size_t)ns * M * P * esz > part_cap) --ns;
    return std::max(ns, 1);
}

// A lone launch with few tiles (coarse levels) would leave most CUs idle
// while its last row tile walks the whole K range, so its K range is split
// over several blocks until the launch has about `target` work items.
static Geo geometry(int mode, int M, int P, int K, int off, int ncoef, size_t part_cap, const TileKnobs &kn)
{
    Geo g = tiles(mode, M, P, kn);
    const long T = (long)g.tiles_m * g.tiles_n;
    const int nk = tile_steps(K, off, ncoef, g.BM, g.BK, g.tiles_m - 1);
    const long target = kn.split_target > 0 ? kn.split_target
                        : (g.kind == 0) ? 8192 : (g.kind == 3) ? 1024 : 2048;
    int ns = 1;
    if (T < target) {
        ns = (int)((target + T - 1) / T);
        ns = std::min(ns, 64);
        ns = std::min(ns, std::max(1, nk / 8));
    }
    g.nsplit = split_cap(mode, M, P, ns, part_cap);
    g.part_bytes = g.nsplit > 1 ? (size_t)g.nsplit * M * P * ((mode == GM_F64) ? 8 : 4) : 0;
    return g;
}

size_t splitk_bytes(int mode, int M, int P, int K, int off, int ncoef, const TileKnobs &kn)
{
    return geometry(mode, M, P, K, off, ncoef, (size_t)-1, kn).part_bytes;
}

static inline long blocks_for(long total)
{
    long b = (total + kThreads - 1) / kThreads;
    return std::max(1L, std::min(b, 65536L));
}

// One grouped launch of Op over the argument sets v (blocks[i] blocks each).
template <class Op>
static hipError_t launch_group(const std::vector<typename Op::A> &v, const std::vector<long> &blocks,
                               Staging *st, hipStream_t s)
{
    using A = typename Op::A;
    if (v.empty()) return hipSuccess;
    if (v.size() > 1 && !st) {   // no staging area: one launch per set
        for (size_t i = 0; i < v.size(); ++i) {
            hipError_t e = launch_group<Op>({v[i]}, {blocks[i]}, nullptr, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    Grp<A> g{};
    long total = 0;
    if (v.size() == 1) {
        if (st && st->record) return hipSuccess;
        g.one = v[0];
        g.n = 1;
        total = blocks[0];
    } else {
        if (!st) return hipErrorInvalidValue;
        std::vector<int> start(v.size() + 1, 0);
        for (size_t i = 0; i < v.size(); ++i) start[i + 1] = start[i] + (int)blocks[i];
        const void *dm = st->put(v.data(), sizeof(A) * v.size());
        const void *ds = st->put(start.data(), sizeof(int) * start.size());
        if (st->record) return hipSuccess;
        g.one = v[0];
        g.many = (const A *)dm;
        g.start = (const int *)ds;
        g.n = (int)v.size();
        total = start.back();
    }
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_group<Op>, dim3((unsigned)total), dim3(kThreads), 0, s, g);
    return hipGetLastError();
}

template <int MODE, int EPI>
static void launch_product_kernel(int kind, const KGrp &g, unsigned blocks, hipStream_t s)
{
    if constexpr (MODE == GM_BF16X3) {
        hipLaunchKernelGGL((k_toep_bf16x3<EPI>), dim3(blocks), dim3(256), 0, s, g);
    } else {
        if (kind == 0) hipLaunchKernelGGL((k_toep_narrow<MODE, EPI>), dim3(blocks), dim3(256), 0, s, g);
        else if (kind == 2) hipLaunchKernelGGL((k_toep_wide<MODE, EPI, 1>), dim3(blocks), dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_toep_wide<MODE, EPI, 0>), dim3(blocks), dim3(256), 0, s, g);
    }
}

// Products of one (mode, epilogue, kernel) class: one launch, plus one
// grouped reduce launch for the products whose K range is split.
template <int MODE, int EPI>
static hipError_t launch_class(std::vector<KP> &kps, const std::vector<Geo> &geos, Staging *st, hipStream_t s)
{
    using PT = typename std::conditional<MODE == GM_F64, double, float>::type;
    if (kps.size() > 1 && !st) {   // no staging area: one launch per product
        for (size_t i = 0; i < kps.size(); ++i) {
            std::vector<KP> one{kps[i]};
            hipError_t e = launch_class<MODE, EPI>(one, {geos[i]}, nullptr, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int kind = geos[0].kind;
    KGrp g{};
    long total = 0;
    if (kps.size() == 1) {
        if (st && st->record) return hipSuccess;
        g.one = kps[0];
        g.n = 1;
        total = (long)kps[0].tiles_m * kps[0].tiles_n * kps[0].nsplit;
    } else {
        if (!st) return hipErrorInvalidValue;
        // work items of every product with their K extent, longest first
        struct It { int steps, p, b; };
        std::vector<It> items;
        for (size_t p = 0; p < kps.size(); ++p) {
            const KP &kp = kps[p];
            const Geo &ge = geos[p];
            const long nitems = (long)kp.tiles_m * kp.tiles_n * kp.nsplit;
            for (long b = 0; b < nitems; ++b) {
                const long t = b / kp.nsplit;
                const int sidx = (int)(b - t * kp.nsplit);
                const int tm = kp.tiles_m - 1 - (int)(t / kp.tiles_n);
                const int nk = tile_steps(kp.K, kp.off, kp.ncoef, ge.BM, ge.BK, tm);
                const int st0 = (int)((long)nk * sidx / kp.nsplit), st1 = (int)((long)nk * (sidx + 1) / kp.nsplit);
                items.push_back({st1 - st0, (int)p, (int)b});
            }
        }
        std::stable_sort(items.begin(), items.end(), [](const It &x, const It &y) { return x.steps > y.steps; });
        std::vector<int2> tab(items.size());
        for (size_t i = 0; i < items.size(); ++i) tab[i] = make_int2(items[i].p, items[i].b);
        const void *dk = st->put(kps.data(), sizeof(KP) * kps.size());
        const void *di = st->put(tab.data(), sizeof(int2) * tab.size());
        total = (long)tab.size();
        if (!st->record) {
            g.one = kps[0];
            g.many = (const KP *)dk;
            g.items = (const int2 *)di;
            g.n = (int)kps.size();
        }
    }
    std::vector<KP> red;
    std::vector<long> rblocks;
    for (const KP &kp : kps)
        if (kp.nsplit > 1) {
            red.push_back(kp);
            rblocks.push_back(blocks_for((long)kp.M * kp.P));
        }
    if (!(st && st->record) && total > 0) launch_product_kernel<MODE, EPI>(kind, g, (unsigned)total, s);
    if (!red.empty()) {
        hipError_t e = launch_group<OpReduce<EPI, PT>>(red, rblocks, st, s);
        if (e != hipSuccess) return e;
    }
    return (st && st->record) ? hipSuccess : hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(int epi, std::vector<KP> &kps, const std::vector<Geo> &geos, Staging *st,
                              hipStream_t s)
{
    switch (epi) {
    case EPI_STORE: return launch_class<MODE, EPI_STORE>(kps, geos, st, s);
    case EPI_SUB: return launch_class<MODE, EPI_SUB>(kps, geos, st, s);
    }
    if constexpr (MODE == GM_F64) {
        if (epi == EPI_SCATTER) return launch_class<MODE, EPI_SCATTER>(kps, geos, st, s);
    } else {
        if (epi == EPI_ADD) return launch_class<MODE, EPI_ADD>(kps, geos, st, s);
    }
    return hipErrorInvalidValue;
}

static hipError_t launch_toep_fft(const std::vector<const GemmArgs *> &all, Staging *st, hipStream_t s);

hipError_t launch_toep_gemm(const std::vector<GemmArgs> &as, Staging *st, hipStream_t s)
{
    // classes of (mode, epilogue, kernel); one launch each
    std::map<int, std::vector<size_t>> cls;
    std::vector<const GemmArgs *> ffts;
    std::vector<Geo> geo(as.size());
    for (size_t i = 0; i < as.size(); ++i) {
        const GemmArgs &a = as[i];
        if (a.M <= 0 || a.P <= 0) continue;
        if (a.fft_spec) {   // FFT route: grouped below
            ffts.push_back(&a);
            continue;
        }
        geo[i] = geometry(a.mode, a.M, a.P, a.K, a.off, a.coef->n, a.part ? a.part_cap : 0, a.knobs);
        cls[(a.mode << 8) | (a.epi << 4) | geo[i].kind].push_back(i);
    }
    RET_IF(launch_toep_fft(ffts, st, s));
    for (auto &kv : cls) {
        const std::vector<size_t> &idx = kv.second;
        std::vector<KP> kps;
        std::vector<Geo> geos;
        if (idx.size() > 1) {
            // a group: the launch is as long as its total work over the
            // concurrent blocks or its longest item, whichever is larger, so
            // split only the products whose longest tile exceeds that share
            const Geo &g0 = geo[idx[0]];
            const double slots = (g0.kind == 0) ? 1024.0 : (g0.kind == 3) ? 256.0 : 512.0;
            double work = 0;
            std::vector<int> longest(idx.size());
            for (size_t j = 0; j < idx.size(); ++j) {
                const GemmArgs &a = as[idx[j]];
                Geo g = tiles(a.mode, a.M, a.P, a.knobs);
                for (int tm = 0; tm < g.tiles_m; ++tm)
                    work += (double)tile_steps(a.K, a.off, a.coef->n, g.BM, g.BK, tm) * g.tiles_n;
                longest[j] = tile_steps(a.K, a.off, a.coef->n, g.BM, g.BK, g.tiles_m - 1);
            }
            const double share = std::max(1.0, work / slots);
            for (size_t j = 0; j < idx.size(); ++j) {
                const GemmArgs &a = as[idx[j]];
                Geo g = tiles(a.mode, a.M, a.P, a.knobs);
                int ns = (int)std::ceil(longest[j] / share);
                ns = std::min(ns, std::min(64, std::max(1, longest[j] / 8)));
                g.nsplit = split_cap(a.mode, a.M, a.P, ns, a.part ? a.part_cap : 0);
                geo[idx[j]] = g;
            }
        }
        for (size_t i : idx) {
            const GemmArgs &a = as[i];
            const Geo &g = geo[i];
            KP kp{};
            kp.M = a.M; kp.P = a.P; kp.K = a.K; kp.off = a.off; kp.ncoef = a.coef->n;
            kp.tiles_m = g.tiles_m; kp.tiles_n = g.tiles_n; kp.nsplit = g.nsplit;
            kp.coef = (a.mode == GM_F64) ? (const void *)a.coef->d64 : (const void *)a.coef->d32;
            kp.fhi = a.coef->fhi; kp.flo = a.coef->flo;
            kp.B = a.B; kp.Bhi = (const uint16_t *)a.Bhi; kp.Blo = (const uint16_t *)a.Blo; kp.ldb = a.ldb;
            kp.part = a.part;
            kp.ea = a.ea;
            kps.push_back(kp);
            geos.push_back(g);
        }
        const int mode = kv.first >> 8, epi = (kv.first >> 4) & 15;
        hipError_t e = hipErrorInvalidValue;
        if (mode == GM_F64) e = launch_mode<GM_F64>(epi, kps, geos, st, s);
        else if (mode == GM_F32) e = launch_mode<GM_F32>(epi, kps, geos, st, s);
        else if (mode == GM_BF16X3) e = launch_mode<GM_BF16X3>(epi, kps, geos, st, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int product_kernel_kind(int mode, int M, int P, const TileKnobs &kn)
{
    return tiles(mode, M, P, kn).kind;
}

// ---------------------------------------------------------------------------
// FFT route of the causal Toeplitz product (Section 5.1: a Toeplitz product
// is the leading block of a circulant product of twice the size, applied
// with FFTs).  Two real columns 2q, 2q+1 of B form one complex sequence of
// length L >= 2M (zero padded); its DFT times the DFT of the zero-padded
// coefficients, transformed back, holds the two causal products in its real
// and imaginary parts (first M entries).  Each transform is a sequence of
// Stockham autosort passes of radix R along time: a thread does one R-point
// DFT in registers for one column pair, so the 64 lanes of a wave read and
// write 64 consecutive column pairs per access.  The product with the
// coefficient spectrum is fused into the first inverse pass and the product
// epilogue into the last one.  Arithmetic in FP64 (the FP64 products) or in
// FP32 (the history products of the mixed-precision cycles); the input may
// be FP64 or FP32.
template <typename T> struct Cx;
template <> struct Cx<double> { typedef double v __attribute__((ext_vector_type(2))); };
template <> struct Cx<float> { typedef float v __attribute__((ext_vector_type(2))); };

template <typename C> __device__ inline C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

struct FftPass {
    int L, Q, Ns;          // length, column pairs of this chunk, length of the sub-transforms done
    int b_colour;          // >= 0: product column j reads B's point colour_point(j)
    int M, K, P, c0;       // output rows, input rows, columns, first column of this chunk
    const void *src;       // complex [L][Q]
    void *dst;             // complex [L][Q]
    const void *B;         // real input [K][ldb] (FP64 or FP32)
    long ldb;
    const void *spec;      // complex [L]
    const void *tw;        // complex [Ltw], exp(-2 pi i k / Ltw)
    int Ltw;
    double scale;          // 1 / L (last inverse pass)
    EpiArgs ea;
};
// The work arrays are read once and written once per pass: their loads and
// stores are nontemporal (measured a few per cent faster).
// FS_RHS: the real input is the smoother's right-hand side computed where it
// is read (rhs_val; FP64 route of a split level).
enum FftSrc { FS_REAL = 0, FS_CPLX = 1, FS_SPEC = 2, FS_RHS = 3 };

// Column of B read for product column j (the colour's points when b_colour >= 0).
__device__ inline int fft_bcol(const FftPass &a, int j)
{
    return a.b_colour < 0 ? j : colour_point(a.ea.dims, a.ea.n, a.b_colour, j);
}
enum FftDst { FD_CPLX = 0, FD_EPI = 1 };

// cos and sin of 2 pi i / 32, i < 32, at compile time: Taylor series on
// [0, pi/4] (14 terms: the remainder is far below the rounding of a double)
// and the symmetries of the circle for the other octants.
constexpr double kPi = 3.14159265358979323846;
constexpr double cx_sin_red(double x)
{
    double x2 = x * x, term = x, sum = x;
    for (int n = 1; n < 14; ++n) {
        term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double cx_cos_red(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int n = 1; n < 14; ++n) {
        term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}
struct Tw32 {
    double c[32], s[32];
    constexpr Tw32() : c(), s()
    {
        for (int i = 0; i < 32; ++i) {
            const int qd = i / 8, r = i % 8;
            double cr = 0.0, sr = 0.0;   // angle r pi / 16 in [0, pi / 2)
            if (r <= 4) {
                cr = cx_cos_red(r * kPi / 16);
                sr = cx_sin_red(r * kPi / 16);
            } else {
                cr = cx_sin_red((8 - r) * kPi / 16);
                sr = cx_cos_red((8 - r) * kPi / 16);
            }
            // rotate by qd quarter turns
            const double cc[4] = {cr, -sr, -cr, sr}, ss[4] = {sr, cr, -sr, -cr};
            c[i] = cc[qd];
            s[i] = ss[qd];
        }
    }
};
constexpr Tw32 kTw32{};

// R-point DFT (R a power of two <= 32) of v in natural order, in registers:
// bit-reversal permutation (register renaming once unrolled), then radix-2
// butterflies with compile-time twiddles; SIGN -1 forward, +1 inverse
// (unnormalised).
template <typename T, int R, int SIGN>
__device__ inline void dft_reg(typename Cx<T>::v (&v)[R])
{
    using C = typename Cx<T>::v;
    constexpr int LG = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : (R == 16) ? 4 : 5;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int j = 0;
#pragma unroll
        for (int b = 0; b < LG; ++b) j |= ((i >> b) & 1) << (LG - 1 - b);
        if (j > i) {
            C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int m = 2; m <= R; m <<= 1) {
#pragma unroll
        for (int t = 0; t < m / 2; ++t) {
            // exp(SIGN 2 pi i t / m); the twiddles 1 and SIGN i (t = 0 and
            // t = m / 4) as a copy and a swap, not as products with zeros
            const int tq = t * (32 / m);
            C w = C{(T)kTw32.c[tq], (T)(SIGN * kTw32.s[tq])};
#pragma unroll
            for (int k = 0; k < R; k += m) {
                const C x = v[k + t + m / 2];
                const C b = (tq == 0) ? x : (tq == 8) ? C{(T)(-SIGN) * x.y, (T)SIGN * x.x} : cmul(x, w);
                const C a = v[k + t];
                v[k + t] = a + b;
                v[k + t + m / 2] = a - b;
            }
        }
    }
}

__device__ inline double nan_max(double a, double m);
__device__ inline void block_reduce(double &mx, double &sq);

template <typename T, typename TIN, int R, int SIGN, int SRC, int DST, int EPI>
__global__ __launch_bounds__(256) void k_fft_pass(Grp<FftPass> grp)
{
    FftPass a;
    long lb, nb;
    grp_select(grp, a, lb, nb);
    using C = typename Cx<T>::v;
    const long g = lb * 256 + threadIdx.x;
    const int nj = a.L / R;
    if (g >= (long)a.Q * nj) return;
    const int q = (int)(g % a.Q), j = (int)(g / a.Q);
    const GLOBAL C *tw = gview<C>(a.tw);
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int tau = j + r * nj;
        if constexpr (SRC == FS_REAL || SRC == FS_RHS) {
            T re = 0, im = 0;
            if (tau < a.K) {
                if constexpr (SRC == FS_RHS) {
                    if (a.c0 + 2 * q < a.P) re = (T)rhs_val(a.ea, tau, a.c0 + 2 * q);
                    if (a.c0 + 2 * q + 1 < a.P) im = (T)rhs_val(a.ea, tau, a.c0 + 2 * q + 1);
                } else {
                    const GLOBAL TIN *row = gview<TIN>(a.B) + (long)tau * a.ldb;
                    if (a.c0 + 2 * q < a.P) re = (T)row[fft_bcol(a, a.c0 + 2 * q)];
                    if (a.c0 + 2 * q + 1 < a.P) im = (T)row[fft_bcol(a, a.c0 + 2 * q + 1)];
                }
            }
            v[r] = C{re, im};
        } else {
            v[r] = __builtin_nontemporal_load(&gview<C>(a.src)[(long)tau * a.Q + q]);
            if constexpr (SRC == FS_SPEC) v[r] = cmul(v[r], gview<C>(a.spec)[tau]);
        }
    }
    const int jm = j % a.Ns;
    if (a.Ns > 1) {
        // exp(SIGN 2 pi i jm r / (Ns R)) = tw[jm r (Ltw / (Ns R))] (conjugated for SIGN > 0)
        const long step = (long)jm * (a.Ltw / (a.Ns * R));
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[step * r];
            if (SIGN > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
    }
    dft_reg<T, R, SIGN>(v);
    const int base = (j / a.Ns) * a.Ns * R + jm;
    if constexpr (DST == FD_CPLX) {
#pragma unroll
        for (int r = 0; r < R; ++r) __builtin_nontemporal_store(v[r], &gview_rw<C>(a.dst)[(long)(base + r * a.Ns) * a.Q + q]);
    } else {
        // the epilogue in groups of rows: their loads, then their stores
        const int c = a.c0 + 2 * q;
        constexpr int G8 = epi_rows<EPI>(R < 8 ? R : 8);
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += G8) {
            double pre[G8][2];
#pragma unroll
            for (int r = 0; r < G8; ++r) {   // at clamped indices: no load behind a branch
                const int tau = min(base + (r0 + r) * a.Ns, a.M - 1);
                pre[r][0] = epi_pre<EPI>(a.ea, tau, min(c, a.P - 1));
                pre[r][1] = epi_pre<EPI>(a.ea, tau, min(c + 1, a.P - 1));
            }
#pragma unroll
            for (int r = 0; r < G8; ++r) {
                const int tau = base + (r0 + r) * a.Ns;
                if (tau >= a.M) continue;
                if (c < a.P) epi_put<EPI>(a.ea, tau, c, pre[r][0], (double)v[r0 + r].x * a.scale);
                if (c + 1 < a.P) epi_put<EPI>(a.ea, tau, c + 1, pre[r][1], (double)v[r0 + r].y * a.scale);
            }
        }
    }
}

// A Stockham pass of radix R = R1 R2 (64, 128 or 256) by one block for NC
// column pairs: the R-point DFT as two stages (Cooley-Tukey, R = R1 x R2):
// R1-point DFTs over elements R2 apart in registers, twiddles, an exchange
// through LDS, then R2-point DFTs, one DFT per thread (16 NC threads; the
// passes other than the last take R2 = 16, so that every thread has a DFT of
// the first stage, the one that reads the input).  Rows
// of NC pairs are read and written whole: 16 pairs in FP64 (256 bytes), 32
// in FP32 (256 bytes, 7 % faster than 16 on the largest products).  16 pairs
// per block beat 8 (narrow rows) and two DFTs per thread.
template <typename T, int EPI = -1> constexpr int fft_lds_cols()
{
    return sizeof(T) == 4 ? 32 : 16;
}
template <typename T, int EPI = -1> constexpr int fft_lds_threads() { return 16 * fft_lds_cols<T, EPI>(); }

template <typename T, typename TIN, int R1, int R2, int SIGN, int SRC, int DST, int EPI>
__global__ __launch_bounds__((fft_lds_threads<T, DST == FD_EPI ? EPI : -1>())) void k_fft_lds(Grp<FftPass> grp)
{
    FftPass a;
    long lb, nb;
    grp_select(grp, a, lb, nb);
    using C = typename Cx<T>::v;
    constexpr int E = DST == FD_EPI ? EPI : -1;
    constexpr int R = R1 * R2, NC = fft_lds_cols<T, E>(), NT = fft_lds_threads<T, E>();
    static_assert(R2 * NC <= NT && R1 * NC <= NT, "one DFT per thread and stage");
    __shared__ C sh[R * NC];
    const int nj = a.L / R;
    const int qblocks = (a.Q + NC - 1) / NC;
    const int qb = (int)(lb % qblocks), j = (int)(lb / qblocks);
    const int q0 = qb * NC;
    const GLOBAL C *tw = gview<C>(a.tw);
    const int jm = j % a.Ns;
    const long pstep = (long)jm * (a.Ltw / (a.Ns * R));   // twiddles of the pass
    const int wstep = a.Ltw / R;                           // twiddles inside the R-point DFT
    // the block's pass twiddles (exp(-+2 pi i jm r / (Ns R)), r < R) and the
    // inner twiddles (exp(-+2 pi i t / R), t < R), read once into LDS
    __shared__ C twp[R], twi[R];
    const int c = threadIdx.x % NC, r2 = threadIdx.x / NC, q = q0 + c;
    const bool busy = r2 < R2;   // R2 NC jobs for NT >= R2 NC threads
    C v[R1];
#pragma unroll
    for (int r1 = 0; r1 < R1; ++r1) {
        const int r = R2 * r1 + r2, tau = j + r * nj;
        C x = C{0, 0};
        if (busy && q < a.Q) {
            if constexpr (SRC == FS_REAL || SRC == FS_RHS) {
                T re = 0, im = 0;
                if (tau < a.K) {
                    if constexpr (SRC == FS_RHS) {
                        if (a.c0 + 2 * q < a.P) re = (T)rhs_val(a.ea, tau, a.c0 + 2 * q);
                        if (a.c0 + 2 * q + 1 < a.P) im = (T)rhs_val(a.ea, tau, a.c0 + 2 * q + 1);
                    } else {
                        const GLOBAL TIN *row = gview<TIN>(a.B) + (long)tau * a.ldb;
                        if (a.c0 + 2 * q < a.P) re = (T)row[fft_bcol(a, a.c0 + 2 * q)];
                        if (a.c0 + 2 * q + 1 < a.P) im = (T)row[fft_bcol(a, a.c0 + 2 * q + 1)];
                    }
                }
                x = C{re, im};
            } else {
                x = __builtin_nontemporal_load(&gview<C>(a.src)[(long)tau * a.Q + q]);
                if constexpr (SRC == FS_SPEC) x = cmul(x, gview<C>(a.spec)[tau]);
            }
        }
        v[r1] = x;
    }
    for (int t = threadIdx.x; t < R; t += NT) {
        C w = a.Ns > 1 ? tw[pstep * t] : C{1, 0}, wi = tw[(long)t * wstep];
        if (SIGN > 0) {
            w.y = -w.y;
            wi.y = -wi.y;
        }
        twp[t] = w;
        twi[t] = wi;
    }
    __syncthreads();
    if (busy) {
        if (a.Ns > 1) {
#pragma unroll
            for (int r1 = 0; r1 < R1; ++r1)
                if (R2 * r1 + r2 > 0) v[r1] = cmul(v[r1], twp[R2 * r1 + r2]);
        }
        dft_reg<T, R1, SIGN>(v);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) sh[(k1 * R2 + r2) * NC + c] = cmul(v[k1], twi[r2 * k1]);
    }
    __syncthreads();
    const int base = (j / a.Ns) * a.Ns * R + jm;
    // FP64 residual with fused norms: this thread's max |r| and sum r^2
    constexpr bool NORMS = DST == FD_EPI && (EPI == EPI_RESID || EPI == EPI_RESID_DD) && sizeof(T) == 8;
    double nmx = 0.0, nsq = 0.0;
    auto acc_norm = [&](double r) {
        nmx = nan_max(fabs(r), nmx);
        nsq += r * r;
    };
    for (int job = threadIdx.x; job < R1 * NC; job += NT) {
        const int c = job % NC, k1 = job / NC, q = q0 + c;
        C v[R2];
#pragma unroll
        for (int r2 = 0; r2 < R2; ++r2) v[r2] = sh[(k1 * R2 + r2) * NC + c];
        dft_reg<T, R2, SIGN>(v);
        if (q >= a.Q) continue;
        if constexpr (DST == FD_CPLX) {
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2)
                __builtin_nontemporal_store(v[k2], &gview_rw<C>(a.dst)[(long)(base + (k1 + R1 * k2) * a.Ns) * a.Q + q]);
        } else {
            // the epilogue in groups of rows: their loads, then their stores
            const int cc = a.c0 + 2 * q;
            constexpr int CH = epi_rows<EPI>(R2);
            if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_DD || EPI == EPI_RESID_C || EPI == EPI_RESID_R) {
                if (a.ea.dims == 1 && !a.ea.lay_in) {   // natural input; cc < P; cc + 1 may be P
                    // first point of the pair: column cc, or the colour's point cc
                    constexpr bool colr = EPI == EPI_RESID_C || EPI == EPI_RESID_R;
                    const int pt = colr ? colour_point(1, a.ea.n, a.ea.colour, cc) : cc;
#pragma unroll
                    for (int k0 = 0; k0 < R2; k0 += CH) {
                        double pre[CH][2];
#pragma unroll
                        for (int k = 0; k < CH; ++k)
                            resid_pre_pair_1d<EPI == EPI_RESID_DD, colr ? 2 : 1>(
                                a.ea, min(base + (k1 + R1 * (k0 + k)) * a.Ns, a.M - 1), pt, pre[k][0], pre[k][1]);
#pragma unroll
                        for (int k = 0; k < CH; ++k) {
                            const int tau = base + (k1 + R1 * (k0 + k)) * a.Ns;
                            if (tau >= a.M) continue;
                            const double q0 = (double)v[k0 + k].x * a.scale, q1 = (double)v[k0 + k].y * a.scale;
                            epi_put<EPI>(a.ea, tau, cc, pre[k][0], q0);
                            if constexpr (NORMS) acc_norm(pre[k][0] - q0);   // the value stored
                            if (cc + 1 < a.P) {
                                epi_put<EPI>(a.ea, tau, cc + 1, pre[k][1], q1);
                                if constexpr (NORMS) acc_norm(pre[k][1] - q1);
                            }
                        }
                    }
                    continue;
                }
            }
#pragma unroll
            for (int k0 = 0; k0 < R2; k0 += CH) {
                double pre[CH][2];
#pragma unroll
                for (int k = 0; k < CH; ++k) {   // at clamped indices: no load behind a branch
                    const int tau = min(base + (k1 + R1 * (k0 + k)) * a.Ns, a.M - 1);
                    pre[k][0] = epi_pre<EPI>(a.ea, tau, min(cc, a.P - 1));
                    pre[k][1] = epi_pre<EPI>(a.ea, tau, min(cc + 1, a.P - 1));
                }
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int tau = base + (k1 + R1 * (k0 + k)) * a.Ns;
                    if (tau >= a.M) continue;
                    const double q0 = (double)v[k0 + k].x * a.scale, q1 = (double)v[k0 + k].y * a.scale;
                    if (cc < a.P) {
                        epi_put<EPI>(a.ea, tau, cc, pre[k][0], q0);
                        if constexpr (NORMS) acc_norm(pre[k][0] - q0);
                    }
                    if (cc + 1 < a.P) {
                        epi_put<EPI>(a.ea, tau, cc + 1, pre[k][1], q1);
                        if constexpr (NORMS) acc_norm(pre[k][1] - q1);
                    }
                }
            }
        }
    }
    if constexpr (NORMS) {
        if (a.ea.norm_part) {   // a launch-wide choice: every thread reaches the reduction
            block_reduce(nmx, nsq);
            if (threadIdx.x == 0) {
                gview_rw<double>(a.ea.norm_part)[2 * lb] = nmx;
                gview_rw<double>(a.ea.norm_part)[2 * lb + 1] = nsq;
            }
        }
    }
}

// The middle of a product by the FFT route in one kernel: the last forward
// pass (radix 256 = 16 x 16; block j holds rows j + k nj, nj = L / 256),
// the product with the coefficient spectrum, and the first inverse pass.
// That pass's RI-point DFTs (RI = the plan's first radix, no twiddles as
// nothing is combined yet) take rows j' + s L / RI; for j' = j + g nj those
// are rows j + nj (g + G s) of this block, G = 256 / RI, so the block does G
// of them from LDS and writes rows j' RI + t.  One read and one write of the
// work array less per product than the two passes.
template <typename T, int RI>
__global__ __launch_bounds__(fft_lds_threads<T>()) void k_fft_mid(Grp<FftPass> grp)
{
    FftPass a;
    long lb, nb;
    grp_select(grp, a, lb, nb);
    using C = typename Cx<T>::v;
    constexpr int R = 256, NC = fft_lds_cols<T>(), NT = fft_lds_threads<T>(), G = R / RI;
    static_assert(16 * NC == NT, "one radix-256 job per thread");
    __shared__ C sh[R * NC];
    const int nj = a.L / R;
    const int qblocks = (a.Q + NC - 1) / NC;
    const int qb = (int)(lb % qblocks), j = (int)(lb / qblocks);
    const int q0 = qb * NC;
    const GLOBAL C *tw = gview<C>(a.tw);
    const GLOBAL C *src = gview<C>(a.src), *spec = gview<C>(a.spec);
    GLOBAL C *dst = gview_rw<C>(a.dst);
    const int wstep = a.Ltw / R;
    // the block's twiddles and spectrum values, read once into LDS: pass
    // twiddles exp(-2 pi i j r / L), inner twiddles exp(-2 pi i t / 256),
    // spectrum rows j + t nj and the inverse inner twiddles exp(2 pi i t / RI)
    __shared__ C twp[R], twi[R], sp[R], twv[RI > 16 ? RI : 1];
    {   // forward, first stage: 16-point DFTs over r = 16 r1 + r2 after the
        // pass twiddles, then the inner twiddles
        const int c = threadIdx.x % NC, r2 = threadIdx.x / NC, q = q0 + c;
        const long pstep = (long)j * (a.Ltw / a.L);
        C v[16];
#pragma unroll
        for (int r1 = 0; r1 < 16; ++r1) {
            const int r = 16 * r1 + r2;
            v[r1] = q < a.Q ? __builtin_nontemporal_load(&src[(long)(j + r * nj) * a.Q + q]) : C{0, 0};
        }
        for (int t = threadIdx.x; t < R; t += NT) {
            twp[t] = tw[pstep * t];
            twi[t] = tw[(long)t * wstep];
            sp[t] = spec[j + t * nj];
            if constexpr (RI > 16) {
                if (t < RI) {
                    C w = tw[(long)t * (a.Ltw / RI)];
                    w.y = -w.y;
                    twv[t] = w;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r1 = 1; r1 < 16; ++r1) v[r1] = cmul(v[r1], twp[16 * r1 + r2]);
        if (r2 > 0) v[0] = cmul(v[0], twp[r2]);
        dft_reg<T, 16, -1>(v);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) sh[(k1 * 16 + r2) * NC + c] = cmul(v[k1], twi[r2 * k1]);
    }
    __syncthreads();
    {   // forward, second stage: Y[k], k = k1 + 16 k2 (row j + k nj), times the spectrum
        const int c = threadIdx.x % NC, k1 = threadIdx.x / NC;
        C v[16];
#pragma unroll
        for (int r2 = 0; r2 < 16; ++r2) v[r2] = sh[(k1 * 16 + r2) * NC + c];
        dft_reg<T, 16, -1>(v);
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) v[k2] = cmul(v[k2], sp[k1 + 16 * k2]);
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) sh[(k1 + 16 * k2) * NC + c] = v[k2];
    }
    __syncthreads();
    // inverse: group g takes x[s] = Y[g + G s], s < RI, and writes its DFT
    // X[t] to row (j + g nj) RI + t
    if constexpr (RI <= 16) {
        for (int job = threadIdx.x; job < G * NC; job += NT) {
            const int c = job % NC, g = job / NC, q = q0 + c;
            C v[RI];
#pragma unroll
            for (int s2 = 0; s2 < RI; ++s2) v[s2] = sh[(g + G * s2) * NC + c];
            dft_reg<T, RI, 1>(v);
            if (q >= a.Q) continue;
            const long row = (long)(j + g * nj) * RI;
#pragma unroll
            for (int t = 0; t < RI; ++t) __builtin_nontemporal_store(v[t], &dst[(row + t) * a.Q + q]);
        }
    } else {
        // RI = 16 x RI2: 16-point DFTs over s = RI2 s1 + s2 (in place), the
        // inner twiddles, then RI2-point DFTs giving X[k1 + 16 k2]
        constexpr int RI2 = RI / 16;
        for (int job = threadIdx.x; job < G * RI2 * NC; job += NT) {
            const int c = job % NC, s2 = (job / NC) % RI2, g = job / (NC * RI2);
            C v[16];
#pragma unroll
            for (int s1 = 0; s1 < 16; ++s1) v[s1] = sh[(g + G * (RI2 * s1 + s2)) * NC + c];
            dft_reg<T, 16, 1>(v);
#pragma unroll
            for (int k1 = 0; k1 < 16; ++k1) sh[(g + G * (RI2 * k1 + s2)) * NC + c] = cmul(v[k1], twv[s2 * k1]);
        }
        __syncthreads();
        for (int job = threadIdx.x; job < G * 16 * NC; job += NT) {
            const int c = job % NC, k1 = (job / NC) % 16, g = job / (NC * 16), q = q0 + c;
            C v[RI2];
#pragma unroll
            for (int s2 = 0; s2 < RI2; ++s2) v[s2] = sh[(g + G * (RI2 * k1 + s2)) * NC + c];
            dft_reg<T, RI2, 1>(v);
            if (q >= a.Q) continue;
            const long row = (long)(j + g * nj) * RI;
#pragma unroll
            for (int k2 = 0; k2 < RI2; ++k2) __builtin_nontemporal_store(v[k2], &dst[(row + k1 + 16 * k2) * a.Q + q]);
        }
    }
}

// The FFT passes are launched for a group of products at once (the same
// transform length and epilogue: one entry per product, blocks after one
// another, each block finding its product as the grouped bandwidth kernels
// do); without a staging area, one launch per product.
template <typename Launch>
static hipError_t fft_launch(Launch &&launch, const std::vector<FftPass> &ps, const std::vector<long> &blocks,
                             Staging *st)
{
    if (ps.empty()) return hipSuccess;
    if (ps.size() > 1 && !st) {
        for (size_t i = 0; i < ps.size(); ++i) {
            hipError_t e = fft_launch(launch, std::vector<FftPass>{ps[i]}, std::vector<long>{blocks[i]}, nullptr);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    Grp<FftPass> g{};
    long total = 0;
    if (ps.size() == 1) {
        if (st && st->record) return hipSuccess;
        g.one = ps[0];
        g.n = 1;
        total = blocks[0];
    } else {
        std::vector<int> start(ps.size() + 1, 0);
        for (size_t i = 0; i < ps.size(); ++i) start[i + 1] = start[i] + (int)blocks[i];
        const void *dm = st->put(ps.data(), sizeof(FftPass) * ps.size());
        const void *ds = st->put(start.data(), sizeof(int) * start.size());
        if (st->record) return hipSuccess;
        g.one = ps[0];
        g.many = (const FftPass *)dm;
        g.start = (const int *)ds;
        g.n = (int)ps.size();
        total = start.back();
    }
    if (total <= 0) return hipSuccess;
    launch(dim3((unsigned)total), g);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fft_mid(int RI, const std::vector<FftPass> &ps, Staging *st, hipStream_t s)
{
    constexpr int NC = fft_lds_cols<T>(), NT = fft_lds_threads<T>();
    std::vector<long> blocks;
    for (const FftPass &p : ps) blocks.push_back((long)((p.Q + NC - 1) / NC) * (p.L / 256));
    auto go = [&](auto kern) {
        return fft_launch([&](dim3 grid, const Grp<FftPass> &g) { hipLaunchKernelGGL(kern, grid, dim3(NT), 0, s, g); },
                          ps, blocks, st);
    };
    switch (RI) {
    case 2: return go(k_fft_mid<T, 2>);
    case 4: return go(k_fft_mid<T, 4>);
    case 8: return go(k_fft_mid<T, 8>);
    case 16: return go(k_fft_mid<T, 16>);
    case 32: return go(k_fft_mid<T, 32>);
    case 64: return go(k_fft_mid<T, 64>);
    case 128: return go(k_fft_mid<T, 128>);
    default: return go(k_fft_mid<T, 256>);
    }
}

// Radices of the passes for a transform of length L = 2^s.  From L = 512 on:
// the remainder (2^(s mod 8)) first, then radix 256 (two stages through
// LDS), so a length-32768 transform takes two passes; the last inverse pass
// (the one with the epilogue) is radix 256.  Shorter transforms: the
// remainder 2^(s mod 5) first, then radix 32 in registers.
static std::vector<int> fft_plan(int L)
{
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    std::vector<int> r;
    if (L >= 512) {
        if (lg % 8) r.push_back(1 << (lg % 8));
        for (int i = 0; i < lg / 8; ++i) r.push_back(256);
        return r;
    }
    if (lg % 5) r.push_back(1 << (lg % 5));
    for (int i = 0; i < lg / 5; ++i) r.push_back(32);
    return r;
}

// ---------------------------------------------------------------------------
// FFT route with the whole product on chip (FP64, transform lengths
// L = 256 R3, R3 in {4, 8, 16}, i.e. M <= 2048): one block of T = L / 16
// threads per column pair, thread j holding the 16 points j + T s of the
// sequence in registers.  Each transform is three Stockham stages (radix 16,
// 16 and R3; the last one as 16 / R3 DFTs per thread) with LDS exchanges
// between them.  The forward transform's last stage leaves thread j the
// spectrum points j + T s, exactly the points the inverse transform's first
// stage reads, so the product with the coefficient spectrum stays in
// registers, and the inverse transform's last stage leaves the outputs
// j + T s, those below M going to the epilogue.  Global traffic is the
// operand read once and the result written once (the pass route also writes
// and reads two complex work arrays).  Blocks go to the 8 XCDs in turn, so
// block b takes pair (b mod 8) nb / 8 + b / 8: the blocks of one XCD take
// consecutive pairs, whose 16-byte row segments share cache lines in its L2.
constexpr int kChipMaxLg = 12;
// two adjacent doubles, 8-byte aligned (one 16-byte access)
typedef double D2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ inline int chip_pad(int i) { return i + (i >> 4); }   // LDS index (bank spread)

template <int LG, int SIGN>
__device__ inline void chip_transform(Cx<double>::v (&v)[16], Cx<double>::v *X, const Cx<double>::v *Wlo,
                                      const Cx<double>::v *Whi)
{
    using C = Cx<double>::v;
    constexpr int L = 1 << LG, T = L / 16, R3 = L / 256, NB = 16 / R3;
    const int j = threadIdx.x;
    // w^m for m < L (conjugated for the inverse)
    auto tw = [&](int m) {
        C w = cmul(Wlo[m & 63], Whi[m >> 6]);
        if (SIGN > 0) w.y = -w.y;
        return w;
    };
    // stage 1 (sub-transforms of length 1 -> 16): the input points j + T r
    dft_reg<double, 16, SIGN>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) X[chip_pad(16 * j + r)] = v[r];
    __syncthreads();
    // stage 2 (16 -> 256)
    {
        const int k = j & 15;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = X[chip_pad(j + T * r)];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], tw(R3 * r * k));   // exp(SIGN 2 pi i r k / 256)
        dft_reg<double, 16, SIGN>(v);
        __syncthreads();
        const int base = (j >> 4) * 256 + k;
#pragma unroll
        for (int r = 0; r < 16; ++r) X[chip_pad(base + 16 * r)] = v[r];
        __syncthreads();
    }
    // stage 3 (256 -> L): butterflies jj = j + T i; its outputs jj + 256 r
    // are the points j + T (i + NB r)
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int jj = j + T * i;
        C u[R3];
#pragma unroll
        for (int r = 0; r < R3; ++r) u[r] = X[chip_pad(jj + 256 * r)];
#pragma unroll
        for (int r = 1; r < R3; ++r) u[r] = cmul(u[r], tw(r * jj));   // exp(SIGN 2 pi i r jj / L)
        dft_reg<double, R3, SIGN>(u);
#pragma unroll
        for (int r = 0; r < R3; ++r) v[i + NB * r] = u[r];
    }
    __syncthreads();   // X is free again
}

template <int LG, int EPI>
__global__ __launch_bounds__(256) void k_fft_chip(Grp<FftPass> grp)
{
    using C = Cx<double>::v;
    constexpr int L = 1 << LG, T = L / 16;
    static_assert(LG >= 10 && LG <= kChipMaxLg, "L = 1024 .. 4096");
    __shared__ C X[L + L / 16];
    __shared__ C Wlo[64], Whi[L / 64];
    FftPass a;
    long lb, nb;
    grp_select(grp, a, lb, nb);
    const int q = (int)((lb & 7) * (nb >> 3) + (lb >> 3));
    const int c = a.c0 + 2 * q;   // the pair's first product column
    if (c >= a.P) return;         // (whole block)
    const int j = threadIdx.x;
    // w^m = Wlo[m mod 64] Whi[m / 64], w = exp(-2 pi i / L)
    const GLOBAL C *tw = gview<C>(a.tw);
    const long st = a.Ltw / L;
    for (int i = j; i < 64; i += T) Wlo[i] = tw[i * st];
    for (int i = j; i < L / 64; i += T) Whi[i] = tw[i * 64 * st];
    // the pair as one complex sequence, zero from row K on
    const bool two = c + 1 < a.P;
    const long b0 = fft_bcol(a, c), b1 = two ? fft_bcol(a, c + 1) : b0;
    const GLOBAL double *B = gview<double>(a.B);
    // adjacent columns: one 16-byte access per row (8-byte aligned)
    const bool adj = two && b1 == b0 + 1;
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = j + T * r;
        C x = C{0.0, 0.0};
        if (m < a.K) {
            const GLOBAL double *row = B + (long)m * a.ldb;
            if (adj) {
                x = *(const GLOBAL D2u *)(row + b0);
            } else {
                x.x = row[b0];
                if (two) x.y = row[b1];
            }
        }
        v[r] = x;
    }
    __syncthreads();   // the twiddle tables
    chip_transform<LG, -1>(v, X, Wlo, Whi);
    const GLOBAL C *spec = gview<C>(a.spec);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cmul(v[r], spec[j + T * r]);
    chip_transform<LG, 1>(v, X, Wlo, Whi);
    // epilogue: the outputs j + T r below M, loads before stores
    double pre[16][2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {   // at clamped indices: no load behind a branch
        const int m = min(j + T * r, a.M - 1);
        pre[r][0] = epi_pre<EPI>(a.ea, m, c);
        pre[r][1] = epi_pre<EPI>(a.ea, m, two ? c + 1 : c);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = j + T * r;
        if (m >= a.M) continue;
        if (EPI == EPI_STORE && two) {   // the pair's two outputs are adjacent
            *(GLOBAL D2u *)(gview_rw<double>(a.ea.out) + (long)m * a.ea.ldo + c) = v[r] * a.scale;
            continue;
        }
        epi_put<EPI>(a.ea, m, c, pre[r][0], v[r].x * a.scale);
        if (two) epi_put<EPI>(a.ea, m, c + 1, pre[r][1], v[r].y * a.scale);
    }
}

// Whether an FFT-route product takes the on-chip kernel.
bool fft_on_chip(const GemmArgs &a)
{
    return a.mode == GM_F64 && !a.ea.rhs && (a.epi == EPI_STORE || a.epi == EPI_SCATTER) && a.fft_L >= 1024 &&
           a.fft_L <= (1 << kChipMaxLg) && (a.fft_L & (a.fft_L - 1)) == 0 && a.K <= a.fft_L / 2 &&
           a.M <= a.fft_L / 2;
}

template <int LG, int EPI>
static hipError_t launch_fft_chip(const std::vector<const GemmArgs *> &as, Staging *st, hipStream_t s)
{
    std::vector<FftPass> ps;
    std::vector<long> blocks;
    for (const GemmArgs *ap : as) {
        const GemmArgs &a = *ap;
        FftPass p{};
        p.L = a.fft_L; p.Q = (a.P + 1) / 2; p.Ns = 0;
        p.M = a.M; p.K = a.K; p.P = a.P; p.c0 = 0;
        p.B = a.B; p.ldb = a.ldb; p.b_colour = a.b_colour;
        p.spec = a.fft_spec; p.tw = a.fft_tw; p.Ltw = a.fft_Ltw;
        p.scale = 1.0 / a.fft_L;
        p.ea = a.ea;
        ps.push_back(p);
        blocks.push_back((p.Q + 7) / 8 * 8);   // a multiple of 8: every set starts on XCD 0
    }
    return fft_launch(
        [&](dim3 grid, const Grp<FftPass> &g) { hipLaunchKernelGGL((k_fft_chip<LG, EPI>), grid, dim3(1 << (LG - 4)), 0, s, g); },
        ps, blocks, st);
}

static hipError_t launch_fft_chip_all(const std::vector<const GemmArgs *> &as, Staging *st, hipStream_t s)
{
    const GemmArgs &a0 = *as[0];
    const int lg = a0.fft_L == 1024 ? 10 : a0.fft_L == 2048 ? 11 : 12;
    if (a0.epi == EPI_STORE) {
        if (lg == 10) return launch_fft_chip<10, EPI_STORE>(as, st, s);
        if (lg == 11) return launch_fft_chip<11, EPI_STORE>(as, st, s);
        return launch_fft_chip<12, EPI_STORE>(as, st, s);
    }
    if (lg == 10) return launch_fft_chip<10, EPI_SCATTER>(as, st, s);
    if (lg == 11) return launch_fft_chip<11, EPI_SCATTER>(as, st, s);
    return launch_fft_chip<12, EPI_SCATTER>(as, st, s);
}

double fft_work_bytes(const GemmArgs &a)
{
    if (fft_on_chip(a)) return 0.0;
    const std::vector<int> plan = fft_plan(a.fft_L);
    // kernels per product: one per pass, the last forward and the first
    // inverse pass fused when the plan ends in radix 256
    const int kernels = 2 * (int)plan.size() - (plan.back() == 256 ? 1 : 0);
    const double array = (double)a.fft_L * ((a.P + 1) / 2) * (a.mode == GM_F64 ? 16.0 : 8.0);
    return 2.0 * (kernels - 1) * array;
}

long fft_fused_blocks(const GemmArgs &a)
{
    if (!a.fft_spec || a.mode != GM_F64) return 0;
    if (fft_plan(a.fft_L).back() != 256) return 0;
    const long Q = (a.P + 1) / 2;
    if (Q > (long)(a.fft_buf_cap / (16 * (size_t)a.fft_L))) return 0;   // several chunks
    constexpr int NC = fft_lds_cols<double, EPI_RESID>();
    return (Q + NC - 1) / NC * (a.fft_L / 256);
}

template <typename T, typename TIN, int R1, int R2, int SIGN, int SRC, int DST, int EPI>
static hipError_t launch_fft_lds(const std::vector<FftPass> &ps, Staging *st, hipStream_t s)
{
    constexpr int E = DST == FD_EPI ? EPI : -1;
    constexpr int R = R1 * R2, NC = fft_lds_cols<T, E>(), NT = fft_lds_threads<T, E>();
    std::vector<long> blocks;
    for (const FftPass &p : ps) blocks.push_back((long)((p.Q + NC - 1) / NC) * (p.L / R));
    return fft_launch(
        [&](dim3 grid, const Grp<FftPass> &g) {
            hipLaunchKernelGGL((k_fft_lds<T, TIN, R1, R2, SIGN, SRC, DST, EPI>), grid, dim3(NT), 0, s, g);
        },
        ps, blocks, st);
}

template <typename T, typename TIN, int SIGN, int SRC, int DST, int EPI>
static hipError_t launch_fft_pass(int R, const std::vector<FftPass> &ps, Staging *st, hipStream_t s)
{
    if (R >= 64) {
        if constexpr (DST == FD_CPLX) {
            if (R == 64) return launch_fft_lds<T, TIN, 4, 16, SIGN, SRC, DST, EPI>(ps, st, s);
            if (R == 128) return launch_fft_lds<T, TIN, 8, 16, SIGN, SRC, DST, EPI>(ps, st, s);
            return launch_fft_lds<T, TIN, 16, 16, SIGN, SRC, DST, EPI>(ps, st, s);
        }
        return hipErrorInvalidValue;
    }
    std::vector<long> blocks;
    for (const FftPass &p : ps) blocks.push_back(((long)p.Q * (p.L / R) + 255) / 256);
    auto go = [&](auto kern) {
        return fft_launch([&](dim3 grid, const Grp<FftPass> &g) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, g); },
                          ps, blocks, st);
    };
    switch (R) {
    case 2: return go(k_fft_pass<T, TIN, 2, SIGN, SRC, DST, EPI>);
    case 4: return go(k_fft_pass<T, TIN, 4, SIGN, SRC, DST, EPI>);
    case 8: return go(k_fft_pass<T, TIN, 8, SIGN, SRC, DST, EPI>);
    case 16: return go(k_fft_pass<T, TIN, 16, SIGN, SRC, DST, EPI>);
    default: return go(k_fft_pass<T, TIN, 32, SIGN, SRC, DST, EPI>);
    }
}

template <typename T, int EPI>
static hipError_t launch_fft_last(int R, const std::vector<FftPass> &ps, Staging *st, hipStream_t s)
{
    if (R == 256) return launch_fft_lds<T, T, 16, 16, 1, FS_CPLX, FD_EPI, EPI>(ps, st, s);
    if (R != 32) return hipErrorInvalidValue;
    std::vector<long> blocks;
    for (const FftPass &p : ps) blocks.push_back(((long)p.Q * (p.L / 32) + 255) / 256);
    return fft_launch(
        [&](dim3 grid, const Grp<FftPass> &g) {
            hipLaunchKernelGGL((k_fft_pass<T, T, 32, 1, FS_CPLX, FD_EPI, EPI>), grid, dim3(256), 0, s, g);
        },
        ps, blocks, st);
}

// Products of one group (the same transform length, arithmetic and
// epilogue), each in one chunk of columns starting at c0[i]: every pass is
// one launch over all of them.
template <typename T, typename TIN>
static hipError_t fft_group(const std::vector<const GemmArgs *> &as, const std::vector<long> &c0, Staging *st,
                            hipStream_t s)
{
    const GemmArgs &a0 = *as[0];
    const std::vector<int> plan = fft_plan(a0.fft_L);
    if (plan.size() < 2) return hipErrorInvalidValue;
    const size_t n = plan.size(), m = as.size();
    std::vector<FftPass> ps(m);
    for (size_t k = 0; k < m; ++k) {
        const GemmArgs &a = *as[k];
        const long qcap = (long)(a.fft_buf_cap / (2 * sizeof(T) * (size_t)a.fft_L));
        FftPass &p = ps[k];
        p.L = a.fft_L;
        p.Q = (int)std::min(qcap, (long)(a.P - c0[k] + 1) / 2);
        p.M = a.M; p.K = a.K; p.P = a.P; p.c0 = (int)c0[k];
        p.B = a.B; p.ldb = a.ldb; p.b_colour = a.b_colour;
        p.spec = a.fft_spec; p.tw = a.fft_tw; p.Ltw = a.fft_Ltw;
        p.scale = 1.0 / a.fft_L;
        p.ea = a.ea;
    }
    int cur = 0;   // buffer the next pass writes (each product has its own two)
    auto to = [&]() { for (size_t k = 0; k < m; ++k) ps[k].dst = cur ? as[k]->fft_buf1 : as[k]->fft_buf0; };
    auto from = [&]() { for (size_t k = 0; k < m; ++k) ps[k].src = ps[k].dst; cur ^= 1; };
    auto ns = [&](int v) { for (FftPass &p : ps) p.Ns = v; };
    // a plan that ends in radix 256 (L >= 512) does its last forward pass,
    // the spectrum and its first inverse pass in one kernel
    const bool mid = plan.back() == 256;
    // forward transform
    int Ns = 1;
    for (size_t i = 0; i + (mid ? 1 : 0) < n; ++i) {
        ns(Ns);
        to();
        if (i == 0 && a0.ea.rhs) {
            if constexpr (std::is_same<T, double>::value) RET_IF((launch_fft_pass<T, TIN, -1, FS_RHS, FD_CPLX, 0>(plan[i], ps, st, s)));
            else return hipErrorInvalidValue;   // right-hand sides computed in the pass: FP64 route only
        } else {
            RET_IF((i == 0 ? launch_fft_pass<T, TIN, -1, FS_REAL, FD_CPLX, 0>(plan[i], ps, st, s)
                           : launch_fft_pass<T, T, -1, FS_CPLX, FD_CPLX, 0>(plan[i], ps, st, s)));
        }
        from();
        Ns *= plan[i];
    }
    size_t i0 = 0;
    if (mid) {
        ns(Ns);
        to();
        RET_IF(launch_fft_mid<T>(plan[0], ps, st, s));
        from();
        i0 = 1;
    }
    // times the coefficient spectrum (unless done), inverse transform, epilogue
    Ns = mid ? plan[0] : 1;
    for (size_t i = i0; i < n; ++i) {
        ns(Ns);
        if (i + 1 < n) {
            to();
            RET_IF((i == 0 ? launch_fft_pass<T, T, 1, FS_SPEC, FD_CPLX, 0>(plan[i], ps, st, s)
                           : launch_fft_pass<T, T, 1, FS_CPLX, FD_CPLX, 0>(plan[i], ps, st, s)));
            from();
        } else {
            switch (a0.epi) {
            case EPI_STORE: RET_IF((launch_fft_last<T, EPI_STORE>(plan[i], ps, st, s))); break;
            case EPI_SCATTER: RET_IF((launch_fft_last<T, EPI_SCATTER>(plan[i], ps, st, s))); break;
            case EPI_RESID: RET_IF((launch_fft_last<T, EPI_RESID>(plan[i], ps, st, s))); break;
            case EPI_RESID_DD: RET_IF((launch_fft_last<T, EPI_RESID_DD>(plan[i], ps, st, s))); break;
            case EPI_RESID_C: RET_IF((launch_fft_last<T, EPI_RESID_C>(plan[i], ps, st, s))); break;
            case EPI_RESID_R: RET_IF((launch_fft_last<T, EPI_RESID_R>(plan[i], ps, st, s))); break;
            case EPI_STORE_DIAG: RET_IF((launch_fft_last<T, EPI_STORE_DIAG>(plan[i], ps, st, s))); break;
            default: return hipErrorInvalidValue;
            }
        }
        Ns *= plan[i];
    }
    return hipSuccess;
}

// The FFT-route products of one launch stage: grouped by transform length,
// arithmetic and epilogue (in order of first appearance); a product whose
// columns need several chunks of the work arrays runs alone, chunk by chunk.
static hipError_t launch_toep_fft(const std::vector<const GemmArgs *> &all, Staging *st, hipStream_t s)
{
    std::vector<std::pair<long, std::vector<const GemmArgs *>>> groups;
    std::map<int, std::vector<const GemmArgs *>> chip;   // on-chip products by (L, epilogue)
    for (const GemmArgs *a : all) {
        if (a->off != 0 || a->K > a->M || a->fft_L < 2 * a->M || a->fft_L < 64 || a->fft_L > a->fft_Ltw)
            return hipErrorInvalidValue;
        if (fft_on_chip(*a)) {
            chip[(a->fft_L << 4) | a->epi].push_back(a);
            continue;
        }
        const size_t csz = (a->mode == GM_F64) ? 16 : 8;
        const long qcap = (long)(a->fft_buf_cap / (csz * (size_t)a->fft_L));
        if (qcap < 1) return hipErrorInvalidValue;
        const long key = ((long)a->fft_L << 8) | (a->mode << 6) | ((a->fft_b64 ? 1 : 0) << 5) |
                         ((a->ea.rhs ? 1 : 0) << 4) | a->epi;
        if ((a->P + 1) / 2 > qcap) {   // several chunks: alone
            groups.push_back({-1, {a}});
            continue;
        }
        // (products of one group must not share work arrays)
        auto fits = [&](const std::vector<const GemmArgs *> &v) {
            for (const GemmArgs *b : v)
                if (b->fft_buf0 == a->fft_buf0) return false;
            return true;
        };
        size_t g = 0;
        while (g < groups.size() && !(groups[g].first == key && fits(groups[g].second))) ++g;
        if (g == groups.size()) groups.push_back({key, {}});
        groups[g].second.push_back(a);
    }
    for (auto &kv : groups) {
        const auto &as = kv.second;
        const GemmArgs &a0 = *as[0];
        auto run = [&](const std::vector<long> &c0) -> hipError_t {
            if (a0.mode == GM_F64) return fft_group<double, double>(as, c0, st, s);
            // FP32 arithmetic (the history products of the mixed cycles) on FP64 or FP32 input
            if (a0.fft_b64) return fft_group<float, double>(as, c0, st, s);
            return fft_group<float, float>(as, c0, st, s);
        };
        if (kv.first >= 0) {
            RET_IF(run(std::vector<long>(as.size(), 0)));
        } else {
            const size_t csz = (a0.mode == GM_F64) ? 16 : 8;
            const long qcap = (long)(a0.fft_buf_cap / (csz * (size_t)a0.fft_L));
            for (long c = 0; c < a0.P; c += 2 * qcap) RET_IF(run({c}));
        }
    }
    for (auto &kv : chip) RET_IF(launch_fft_chip_all(kv.second, st, s));
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Colour right-hand side of the smoother (Section 3, eq. red-black; Section 6,
// eq. red-black_2d): b = f + c d g + (neighbour sum) / h^2 at the points of
// one colour, gathered into a dense panel (the B operand of the product).
template <typename S> struct OpRhsPanel {
    using A = RhsArgs;
    __device__ static void run(const RhsArgs &a, long lb, long nb)
    {
        const int Pc = colour_count(a.dims, a.n, a.colour);
        const long P = (a.dims == 1) ? a.n : (long)a.n * a.n;
        GLOBAL S *panel = gview_rw<S>(a.panel);
        const GLOBAL double *F = gview<double>(a.F), *cd = gview<double>(a.cd), *g = gview<double>(a.g);
        GLOBAL double *U = gview_rw<double>(a.U);
        for (KsWalk w(lb, nb, Pc); w.k < a.M; w.next()) {
            const long k = w.k;
            const int j = w.s;
            int x = 0, y = 0, pt;   // natural index pt (x + n y in 2D)
            if (a.dims == 2) {
                colour_xy(a.n, a.colour, j, x, y);
                pt = y * a.n + x;
            } else {
                pt = colour_point(1, a.n, a.colour, j);
            }
            const int sp = a.split ? lay_cpos(a.dims, a.n, 1, a.colour, j) : pt;   // stored at
            GLOBAL double *Uk = U + k * P;
            const double ns = a.zero_nbrs ? 0.0
                              : (a.dims == 2) ? nbr_sum_xy(Uk, a.n, x, y, a.split) : nbr_sum(Uk, 1, a.n, pt, a.split);
            double b = F[k * P + sp] + ns * a.ih2;
            if (a.g) b += cd[k] * g[pt];
            panel[(long)k * a.ldp + j] = (S)b;
            if (a.lam0 != 0.0) Uk[sp] = a.lam0 * b;
        }
    }
};

__device__ inline void store_split8(const float *b, void *hi, void *lo, long e)
{
    uint16_t h8[8], l8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint16_t hb = f2bf(b[q]);
        h8[q] = hb;
        l8[q] = f2bf(b[q] - bf2f(hb));
    }
    u32x4 vh, vl;
    vh.x = h8[0] | ((uint32_t)h8[1] << 16); vh.y = h8[2] | ((uint32_t)h8[3] << 16);
    vh.z = h8[4] | ((uint32_t)h8[5] << 16); vh.w = h8[6] | ((uint32_t)h8[7] << 16);
    vl.x = l8[0] | ((uint32_t)l8[1] << 16); vl.y = l8[2] | ((uint32_t)l8[3] << 16);
    vl.z = l8[4] | ((uint32_t)l8[5] << 16); vl.w = l8[6] | ((uint32_t)l8[7] << 16);
    gview_rw<u32x4>(hi)[e] = vh;
    gview_rw<u32x4>(lo)[e] = vl;
}

// Same right-hand side as split BF16 hi/lo in the k8-packed layout
// [Mpad/8][ldp][8] (zero outside k < M, j < Pc).  One thread builds the 8
// time rows of one column.
struct OpRhsPacked {
    using A = RhsArgs;
    __device__ static void run(const RhsArgs &a, long lb, long nb)
    {
        const int Pc = colour_count(a.dims, a.n, a.colour);
        const long P = (a.dims == 1) ? a.n : (long)a.n * a.n;
        const GLOBAL double *F = gview<double>(a.F), *cd = gview<double>(a.cd), *g = gview<double>(a.g);
        GLOBAL double *U = gview_rw<double>(a.U);
        for (KsWalk w(lb, nb, (int)a.ldp); w.k < a.Mpad / 8; w.next()) {
            const int kg = (int)w.k, j = w.s;
            const long e = w.k * a.ldp + j;
            float b8[8];
            // the point: natural index pt (x + n y in 2D), storage index sp
            int x = 0, y = 0, pt = 0, sp = 0;
            if (j < Pc) {
                if (a.dims == 2) {
                    colour_xy(a.n, a.colour, j, x, y);
                    pt = y * a.n + x;
                } else {
                    pt = colour_point(1, a.n, a.colour, j);
                }
                sp = a.split ? lay_cpos(a.dims, a.n, 1, a.colour, j) : pt;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int k = kg * 8 + q;
                double b = 0.0;
                if (k < a.M && j < Pc) {
                    GLOBAL double *Uk = U + (long)k * P;
                    const double ns = a.zero_nbrs ? 0.0
                                      : (a.dims == 2) ? nbr_sum_xy(Uk, a.n, x, y, a.split)
                                                      : nbr_sum(Uk, 1, a.n, pt, a.split);
                    b = F[(long)k * P + sp] + ns * a.ih2;
                    if (a.g) b += cd[k] * g[pt];
                    if (a.lam0 != 0.0) Uk[sp] = a.lam0 * b;
                }
                b8[q] = (float)b;
            }
            store_split8(b8, a.panel, a.panel_lo, e);
        }
    }
};

// Residual (Section 2, eq. discrete_model_IVP_1; Section 6) from the Toeplitz
// product already stored in out: out = (f + c d g - diag u - A_h u) - out.
// With lo != nullptr the iterate is the double-double hi + lo and A_h is
// applied with error-free transformations.
struct OpPost {
    using A = PostArgs;
    __device__ static void run(const PostArgs &a, long lb, long nb)
    {
        const int n = a.n, P = (a.dims == 1) ? n : n * n;
        const GLOBAL double *F = gview<double>(a.F), *U = gview<double>(a.U), *lo = gview<double>(a.lo);
        const GLOBAL double *cd = gview<double>(a.cd), *g = gview<double>(a.g);
        GLOBAL double *out = gview_rw<double>(a.out);
        const GLOBAL double *prod = a.prod ? gview<double>(a.prod) : out;
        for (KsWalk w(lb, nb, P); w.k < a.M; w.next()) {
            // s: storage index (order lay_in), p = x + n y: the natural point
            const int k = (int)w.k, s = w.s;
            const long e = (long)k * P + s;
            int x, y;
            if (a.dims == 2) lay_xy(n, a.lay_in, s, x, y);
            else x = lay_nat(1, n, a.lay_in, s), y = 0;
            const int p = y * n + x;
            const GLOBAL double *Uk = U + (long)k * P;
            double rhs = F[e];
            if (a.g) rhs += cd[k] * g[p];
            if (a.diag != 0.0) rhs -= a.diag * Uk[s];
            double r;
            if (a.lo) {
                double shi, slo;
                if (a.dims == 2) stencil_dd_xy(Uk, lo + (long)k * P, n, x, y, s, shi, slo, a.lay_in);
                else stencil_dd(Uk, lo + (long)k * P, 1, n, p, shi, slo, a.lay_in);
                r = (rhs - shi * a.ih2) - slo * a.ih2;
            } else {
                const double ns = (a.dims == 2) ? nbr_sum_xy(Uk, n, x, y, a.lay_in) : nbr_sum(Uk, 1, n, p, a.lay_in);
                double st = (a.dims == 1 ? 2.0 : 4.0) * Uk[s] - ns;
                r = rhs - st * a.ih2;
            }
            const long o = (a.lay_out == a.lay_in)
                               ? e
                               : (long)k * P + (a.dims == 2 ? lay_pos_xy(n, a.lay_out, x, y) : lay_pos(1, n, a.lay_out, p));
            out[o] = r - prod[e];
        }
    }
};

// Low-precision operands of the products (and the D&C diagonal part).
struct OpOperandF32 {
    using A = OperandArgs;
    __device__ static void run(const OperandArgs &a, long lb, long nb)
    {
        GLOBAL float *out = gview_rw<float>(a.out);
        const GLOBAL double *X = gview<double>(a.X);
        GLOBAL double *X2 = gview_rw<double>(a.X2);
        GRID_STRIDE(e, (long)a.M * a.P) {
            int k = (int)(e / a.P), j = (int)(e - (long)k * a.P);
            double x = X[(long)k * a.ldx + j];
            out[(long)k * a.ldp + j] = (float)x;
            if (a.X2) X2[(long)k * a.ldx + j] = a.s2 * x;
        }
    }
};
struct OpOperandBf16 {
    using A = OperandArgs;
    __device__ static void run(const OperandArgs &a, long lb, long nb)
    {
        const GLOBAL double *X = gview<double>(a.X);
        GLOBAL double *X2 = gview_rw<double>(a.X2);
        GRID_STRIDE(e, (long)(a.Mpad / 8) * a.ldp) {
            int kg = (int)(e / a.ldp), j = (int)(e - (long)kg * a.ldp);
            float b8[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int k = kg * 8 + q;
                double x = 0.0;
                if (k < a.M && j < a.P) {
                    x = X[(long)k * a.ldx + j];
                    if (a.X2) X2[(long)k * a.ldx + j] = a.s2 * x;
                }
                b8[q] = (float)x;
            }
            store_split8(b8, a.out, a.out_lo, e);
        }
    }
};

// Full weighting (Section 3; Section 6): coarse node J on fine node 2J,
// weights [1 2 1]/4 (1D) and their tensor product /16 (2D).  Linear /
// bilinear interpolation of the coarse correction, added to the fine iterate;
// coarse values on the boundary are zero.
__device__ inline double coarse_at(const GLOBAL double *e, int nc, int X)  // X: 1-based coarse index
{
    return (X >= 1 && X <= nc) ? e[X - 1] : 0.0;
}

struct OpXfer {
    using A = XferArgs;
    __device__ static void restrict_fw(const XferArgs &a, long lb, long nb)
    {
        const int nf = a.n, nc = (nf - 1) / 2;
        const int Pc = (a.dims == 1) ? nc : nc * nc;
        const long Pf = (a.dims == 1) ? nf : (long)nf * nf;
        const int sp = a.split;
        for (KsWalk w(lb, nb, Pc); w.k < a.M; w.next()) {
            const long e = w.k * Pc + w.s;
            const GLOBAL double *r = gview<double>(a.src) + w.k * Pf;
            // the coarse point is a colour-0 point of the fine grid, its
            // edge neighbours colour 1, its corners (2D) colour 0; with
            // zero_colour set, that colour's entries are zero and not read
            double v;
            if (a.dims == 1) {
                // q: natural index of the coarse point stored at s (both
                // levels in the order `split`)
                const int q = lay_nat(1, nc, sp, w.s);
                int x = 2 * q + 1;
                auto R = [&](int xx) {
                    return a.implicit ? a.ih2 * nbr_sum(r, 1, nf, xx, sp) : r[lay_pos(1, nf, sp, xx)];
                };
                if (a.zero_colour == 1) v = 0.25 * (2.0 * R(x));
                else if (a.zero_colour == 0) v = 0.25 * (R(x - 1) + R(x + 1));
                else v = 0.25 * (R(x - 1) + 2.0 * R(x) + R(x + 1));
            } else if (a.implicit && a.zero_colour == 1) {
                // the implicit residual at the centre and the four corners,
                // each ih2 times its four second-colour neighbours, weighted
                // 4 and 1: the four edge midpoints enter with weight 6 and the
                // eight second-colour points two apart with weight 1 (zero
                // outside the grid), twelve loads instead of twenty
                int I, J;
                lay_xy(nc, sp, w.s, I, J);
                const int x = 2 * I + 1, y = 2 * J + 1;
                auto at = [&](int yy, int xx) {   // clamped index, zero outside
                    const double v = r[lay_pos_xy(nf, sp, min(max(xx, 0), nf - 1), min(max(yy, 0), nf - 1))];
                    return (xx < 0 || xx >= nf || yy < 0 || yy >= nf) ? 0.0 : v;
                };
                const double inner = (r[lay_pos_xy(nf, sp, x, y - 1)] + r[lay_pos_xy(nf, sp, x, y + 1)]) +
                                     (r[lay_pos_xy(nf, sp, x - 1, y)] + r[lay_pos_xy(nf, sp, x + 1, y)]);
                const double outer = ((at(y - 2, x - 1) + at(y - 2, x + 1)) + (at(y + 2, x - 1) + at(y + 2, x + 1))) +
                                     ((at(y - 1, x - 2) + at(y + 1, x - 2)) + (at(y - 1, x + 2) + at(y + 1, x + 2)));
                v = a.ih2 * (6.0 * inner + outer) * (1.0 / 16.0);
            } else {
                int I, J;
                lay_xy(nc, sp, w.s, I, J);
                int x = 2 * I + 1, y = 2 * J + 1;
                auto R = [&](int yy, int xx) {
                    return a.implicit ? a.ih2 * nbr_sum_xy(r, nf, xx, yy, sp) : r[lay_pos_xy(nf, sp, xx, yy)];
                };
                if (a.zero_colour == 1)
                    v = (R(y - 1, x - 1) + R(y - 1, x + 1) + 2.0 * (2.0 * R(y, x)) + R(y + 1, x - 1) + R(y + 1, x + 1))
                        * (1.0 / 16.0);
                else if (a.zero_colour == 0)
                    v = (2.0 * R(y - 1, x) + 2.0 * (R(y, x - 1) + R(y, x + 1)) + 2.0 * R(y + 1, x)) * (1.0 / 16.0);
                else
                    v = (R(y - 1, x - 1) + 2.0 * R(y - 1, x) + R(y - 1, x + 1)
                         + 2.0 * (R(y, x - 1) + 2.0 * R(y, x) + R(y, x + 1))
                         + R(y + 1, x - 1) + 2.0 * R(y + 1, x) + R(y + 1, x + 1)) * (1.0 / 16.0);
            }
            gview_rw<double>(a.dst)[e] = v;
        }
    }
    __device__ static void prolong_add(const XferArgs &a, long lb, long nb)
    {
        const int nc = a.n, nf = 2 * nc + 1;
        const long Pc = (a.dims == 1) ? nc : (long)nc * nc;
        const long Pf = (a.dims == 1) ? nf : (long)nf * nf;
        const int sp = a.split;
        // with skip_colour, the points of the other colour only
        const int oc = 1 - a.skip_colour;
        const int Pw = a.skip_colour >= 0 ? colour_count(a.dims, nf, oc) : (int)Pf;
        for (KsWalk w(lb, nb, Pw); w.k < a.M; w.next()) {
            const int jw = w.s;
            const GLOBAL double *c = gview<double>(a.src) + w.k * Pc;
            double v;
            long e;   // storage index of the fine point
            if (a.dims == 1) {
                e = w.k * Pf + (a.skip_colour >= 0 ? lay_cpos(1, nf, sp, oc, jw) : jw);
                const int p = a.skip_colour >= 0 ? colour_point(1, nf, oc, jw) : lay_nat(1, nf, sp, jw);
                int nn = p + 1;   // paper numbering
                auto at = [&](int X) -> double { return (X >= 1 && X <= nc) ? c[lay_pos(1, nc, sp, X - 1)] : 0.0; };
                v = 0.5 * (at(nn / 2) + at((nn + 1) / 2));
            } else {
                int x, y;   // the fine point
                if (a.skip_colour >= 0) colour_xy(nf, oc, jw, x, y);
                else lay_xy(nf, sp, jw, x, y);
                e = w.k * Pf + lay_pos_xy(nf, sp, x, y);
                int nn = x + 1, ll = y + 1;
                int xa = nn / 2, xb = (nn + 1) / 2, ya = ll / 2, yb = (ll + 1) / 2;
                auto at = [&](int X, int Y) -> double {
                    return (X >= 1 && X <= nc && Y >= 1 && Y <= nc) ? c[lay_pos_xy(nc, sp, X - 1, Y - 1)] : 0.0;
                };
                v = 0.25 * (at(xa, ya) + at(xb, ya) + at(xa, yb) + at(xb, yb));
            }
            gview_rw<double>(a.dst)[e] += v;
        }
    }
    __device__ static void run(const XferArgs &a, long lb, long nb)
    {
        if (a.dir == 0) restrict_fw(a, lb, nb);
        else prolong_add(a, lb, nb);
    }
};

struct OpFill {
    using A = FillArgs;
    __device__ static void run(const FillArgs &a, long lb, long nb)
    {
        const GLOBAL double *cd = gview<double>(a.cd), *g = gview<double>(a.g);
        GLOBAL double *u = gview_rw<double>(a.u);
        GRID_STRIDE(e, a.M * a.P) {
            double v = 0.0;
            if (a.g) {
                const int p = lay_nat(a.dims, a.n, a.split, (int)(e % a.P));
                v = a.scaled ? cd[e / a.P] * g[p] : g[p];
            }
            u[e] = v;
        }
    }
};

// Deterministic norms: block b of a set reduces a fixed contiguous share
// into partials[b]; one block per set reduces the partials in a fixed order.
// A NaN, once seen, is kept by the max.
__device__ inline double nan_max(double a, double m) { return (a > m || a != a) ? a : m; }

__device__ inline void block_reduce(double &mx, double &sq)
{
    __shared__ double smax[kThreads], ssum[kThreads];
    smax[threadIdx.x] = mx;
    ssum[threadIdx.x] = sq;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smax[threadIdx.x] = nan_max(smax[threadIdx.x + w], smax[threadIdx.x]);
            ssum[threadIdx.x] += ssum[threadIdx.x + w];
        }
        __syncthreads();
    }
    mx = smax[0];
    sq = ssum[0];
}

struct OpNormPartial {
    using A = NormArgs;
    __device__ static void run(const NormArgs &a, long lb, long nb)
    {
        const long per = (a.n + nb - 1) / nb;
        const long beg = lb * per, end = min(a.n, beg + per);
        double mx = 0.0, sq = 0.0;
        const GLOBAL double *x = gview<double>(a.x);
        for (long e = beg + threadIdx.x; e < end; e += kThreads) {
            double v = x[e];
            mx = nan_max(fabs(v), mx);
            sq += v * v;
        }
        block_reduce(mx, sq);
        if (threadIdx.x == 0) {
            gview_rw<double>(a.partials)[2 * lb] = mx;
            gview_rw<double>(a.partials)[2 * lb + 1] = sq;
        }
    }
};

struct OpNormFinal {
    using A = NormArgs;
    __device__ static void run(const NormArgs &a, long, long)
    {
        double mx = 0.0, sq = 0.0;
        const GLOBAL double *part = gview<double>(a.partials);
        for (int b = threadIdx.x; b < a.nblk; b += kThreads) {
            mx = nan_max(part[2 * b], mx);
            sq += part[2 * b + 1];
        }
        block_reduce(mx, sq);
        if (threadIdx.x == 0) {
            gview_rw<double>(a.out2)[0] = mx;
            gview_rw<double>(a.out2)[1] = sqrt(sq);
        }
    }
};

// (hi, lo) <- (hi, lo) + e as a renormalised double-double (TwoSum, then
// fast renormalisation); with lo == nullptr a plain FP64 add.
struct OpDD {
    using A = DDArgs;
    __device__ static void run(const DDArgs &a, long lb, long nb)
    {
        const GLOBAL double *ev = gview<double>(a.e);
        GLOBAL double *hi = gview_rw<double>(a.hi), *lo = gview_rw<double>(a.lo);
        auto add = [&](long i, double d) {
            if (!a.lo) {
                hi[i] += d;
                return;
            }
            double s, err;
            two_sum(hi[i], d, s, err);
            double l = lo[i] + err;
            double h2 = s + l;
            lo[i] = l - (h2 - s);
            hi[i] = h2;
        };
        if (!a.split) {
            GRID_STRIDE(i, a.n) add(i, ev[i]);
            return;
        }
        // e in the storage order `split`: natural point p of row k is at
        // lay_pos of it
        const int n = a.npd, P = (a.dims == 1) ? n : n * n;
        const long rows = a.n / P;
        for (KsWalk w(lb, nb, P); w.k < rows; w.next()) {
            const int p = w.s;
            int sp;
            if (a.dims == 2) {
                const int y = p / n;
                sp = lay_pos_xy(n, 1, p - y * n, y);
            } else {
                sp = lay_pos(1, n, 1, p);
            }
            add(w.k * P + p, ev[w.k * P + sp]);
        }
    }
};

// The D&C solution panel back into the colour's points of the iterate.
struct OpScatter {
    using A = ScatterArgs;
    __device__ static void run(const ScatterArgs &a, long lb, long nb)
    {
        const long P = (a.dims == 1) ? a.n : (long)a.n * a.n;
        const GLOBAL double *X = gview<double>(a.X);
        GLOBAL double *U = gview_rw<double>(a.U);
        GRID_STRIDE(e, (long)a.M * a.Pc) {
            int k = (int)(e / a.Pc), j = (int)(e - (long)k * a.Pc);
            U[(long)k * P + lay_cpos(a.dims, a.n, a.split, a.colour, j)] = X[e];
        }
    }
};

// Between natural order and the split storage order (the refinement's inner
// hierarchy), for the entry points that run its kernels on caller arrays.
struct OpPermute {
    using A = PermuteArgs;
    __device__ static void run(const PermuteArgs &a, long lb, long nb)
    {
        const long P = (a.dims == 1) ? a.n : (long)a.n * a.n;
        const GLOBAL double *src = gview<double>(a.src);
        GLOBAL double *dst = gview_rw<double>(a.dst);
        GRID_STRIDE(e, (long)a.M * P) {
            const long k = e / P;
            const int p = (int)(e - k * P);
            const long q = k * P + lay_pos(a.dims, a.n, 1, p);
            if (a.to_split) dst[q] = src[e];
            else dst[e] = src[q];
        }
    }
};

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
// Launchers: one launch per argument-set type (the right-hand side and the
// operands split by format).
template <class Op, class Pred, class Count>
static hipError_t launch_subset(const std::vector<typename Op::A> &v, Pred pred, Count count, Staging *st,
                                hipStream_t s)
{
    std::vector<typename Op::A> sub;
    std::vector<long> blocks;
    for (const auto &a : v)
        if (pred(a)) {
            sub.push_back(a);
            blocks.push_back(count(a));
        }
    return launch_group<Op>(sub, blocks, st, s);
}

hipError_t launch_rhs(const std::vector<RhsArgs> &v, Staging *st, hipStream_t s)
{
    auto elems = [](const RhsArgs &a) { return blocks_for((long)a.M * colour_count(a.dims, a.n, a.colour)); };
    RET_IF(launch_subset<OpRhsPanel<double>>(v, [](const RhsArgs &a) { return a.fmt == 0; }, elems, st, s));
    RET_IF(launch_subset<OpRhsPanel<float>>(v, [](const RhsArgs &a) { return a.fmt == 1; }, elems, st, s));
    return launch_subset<OpRhsPacked>(
        v, [](const RhsArgs &a) { return a.fmt == 2; },
        [](const RhsArgs &a) { return blocks_for((long)(a.Mpad / 8) * a.ldp); }, st, s);
}

hipError_t launch_post(const std::vector<PostArgs> &v, Staging *st, hipStream_t s)
{
    return launch_subset<OpPost>(
        v, [](const PostArgs &) { return true; },
        [](const PostArgs &a) { return blocks_for((long)a.M * ((a.dims == 1) ? a.n : (long)a.n * a.n)); }, st,
        s);
}

hipError_t launch_operand(const std::vector<OperandArgs> &v, Staging *st, hipStream_t s)
{
    RET_IF(launch_subset<OpOperandF32>(
        v, [](const OperandArgs &a) { return a.fmt == 1; },
        [](const OperandArgs &a) { return blocks_for((long)a.M * a.P); }, st, s));
    return launch_subset<OpOperandBf16>(
        v, [](const OperandArgs &a) { return a.fmt == 2; },
        [](const OperandArgs &a) { return blocks_for((long)(a.Mpad / 8) * a.ldp); }, st, s);
}

hipError_t launch_xfer(const std::vector<XferArgs> &v, Staging *st, hipStream_t s)
{
    return launch_subset<OpXfer>(
        v, [](const XferArgs &) { return true; },
        [](const XferArgs &a) {
            long np = (a.dir == 0) ? (a.n - 1) / 2 : 2 * a.n + 1;
            long pts = (a.dims == 1) ? np : np * np;
            if (a.dir == 1 && a.skip_colour >= 0) pts = colour_count(a.dims, (int)np, 1 - a.skip_colour);
            return blocks_for((long)a.M * pts);
        },
        st, s);
}

hipError_t launch_fill(const std::vector<FillArgs> &v, Staging *st, hipStream_t s)
{
    return launch_subset<OpFill>(
        v, [](const FillArgs &) { return true; }, [](const FillArgs &a) { return blocks_for(a.M * a.P); }, st, s);
}

int norm_partial_blocks(long n)
{
    long b = (n + 8L * kThreads - 1) / (8L * kThreads);
    return (int)std::max(1L, std::min(b, 2048L));
}

hipError_t launch_norms(const std::vector<NormArgs> &v, Staging *st, hipStream_t s)
{
    RET_IF(launch_subset<OpNormPartial>(
        v, [](const NormArgs &a) { return !a.have_partials; }, [](const NormArgs &a) { return (long)a.nblk; }, st, s));
    return launch_subset<OpNormFinal>(
        v, [](const NormArgs &) { return true; }, [](const NormArgs &) { return 1L; }, st, s);
}

hipError_t launch_dd_update(const std::vector<DDArgs> &v, Staging *st, hipStream_t s)
{
    return launch_subset<OpDD>(
        v, [](const DDArgs &) { return true; }, [](const DDArgs &a) { return blocks_for(a.n); }, st, s);
}

hipError_t launch_scatter(const std::vector<ScatterArgs> &v, Staging *st, hipStream_t s)
{
    return launch_subset<OpScatter>(
        v, [](const ScatterArgs &) { return true; },
        [](const ScatterArgs &a) { return blocks_for((long)a.M * a.Pc); }, st, s);
}

hipError_t launch_permute(const std::vector<PermuteArgs> &v, Staging *st, hipStream_t s)
{
    std::vector<long> b;
    for (const auto &a : v) b.push_back(blocks_for((long)a.M * (a.dims == 1 ? a.n : (long)a.n * a.n)));
    return launch_group<OpPermute>(v, b, st, s);
}

hipError_t launch_build_coef(ToepCoef &c, hipStream_t s)
{
    long tot = (long)c.nq * 512 + c.n;
    hipLaunchKernelGGL(k_build_coef, dim3((unsigned)blocks_for(tot)), dim3(kThreads), 0, s, c.n, c.d64, c.d32,
                       c.nq, c.fhi, c.flo);
    return hipGetLastError();
}

}  // namespace mgwr
