// Internal interfaces of the MGWR library: device data layouts and the
// kernel launchers the host runtime (mgwr_capi.cpp) drives.
//
// All grid functions (iterates, right-hand sides, residuals) are FP64 in HBM,
// time-major [M][P].  Only the operands of the Toeplitz products may be held
// in lower precision (FP32 panels, or split-BF16 hi/lo panels in the k8-packed
// layout [Mpad/8][ld][8]).
//
// Every launcher takes a list of per-problem argument sets and issues ONE
// launch for all of them (a batch of independent problems advances stage by
// stage).  A list of one is passed by value in the kernel arguments; longer
// lists go through a Staging area (device copies of the argument arrays).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

namespace mgwr {

// Records msg for mgwr_last_error and returns code.
int set_error(int code, const char *msg);


// Arithmetic of a causal Toeplitz product (history GEMM).
enum GemmMode { GM_F64 = 0, GM_F32 = 1, GM_BF16X3 = 2 };

// BF16 MFMA fragment table of one Toeplitz coefficient vector t[0..n-1].
// Fragment q (q = -kQOff .. nq - kQOff - 1) holds, for lane l and element e,
// t[16 q + (l % 16) - (8 (l / 16) + e)] (zero outside [0, n)): the A operand
// of v_mfma_f32_16x16x32_bf16 for a 16x32 tile whose row/column origins
// differ by 16 q.  hi = bf16(t), lo = bf16(t - hi); 1 KB per fragment each.
constexpr int kQOff = 16;

struct ToepCoef {
    int n = 0;                 // number of coefficients
    double *d64 = nullptr;     // [n]
    float *d32 = nullptr;      // [n]
    uint16_t *fhi = nullptr;   // [nq][64][8]
    uint16_t *flo = nullptr;
    int nq = 0;
};

// Epilogues of the Toeplitz product acc[i][p] = sum_k t[off + i - k] B[k][p].
// They are kept light (one load and one store per element) so that the
// product kernels keep their occupancy; the stencil parts of the residual
// and of the smoother run in the bandwidth kernels before the product.
enum EpiKind {   // the values are part of the kernel ids of the profiling records
    EPI_STORE = 0,       // out[i][p] = acc                        (residual product)
    EPI_SCATTER = 1,     // out[i][colour_point(p)] = acc          (FP64 smoother on a level
                         //   in natural order, full product)
    EPI_SUB = 3,         // out[i][p] -= acc                       (D&C history update)
    EPI_ADD = 4,         // out[i][p] += acc                       (D&C base block, or a
                         //   split level's colour points: the history part)
    EPI_RESID = 6,       // out[i][p] = (F + cd g - diag U - A_h U) - acc at (i, p)  (the
                         //   residual; FFT route only)
    EPI_RESID_DD = 7,    // the same with the iterate U + lo (double-double)
    EPI_RESID_C = 8,     // EPI_RESID at the points of one colour: product column p is
                         //   point colour_point(p) (the other colour's residual is zero
                         //   after a red-black sweep and is neither computed nor written)
    EPI_RESID_R = 9,     // 1D, colour 0: EPI_RESID_C restricted on the fly: colour 0's
                         //   points are the coarse points and the other colour's
                         //   residual is zero, so out[i][p] = 0.25 (2 r) is the coarse
                         //   right-hand side (full weighting)
    EPI_STORE_DIAG = 10  // out[i][p] = diag b[i][p] + acc: the FP64 diagonal term of the
                         //   line solve plus its history product, into the contiguous
                         //   points of one colour of a split level (FP32 FFT route)
};

struct EpiArgs {
    double *out = nullptr;     // output (STORE/SUB/ADD/STORE_DIAG) or the iterate U of the level (SCATTER)
    long ldo = 0;
    int dims = 1, n = 1, colour = 0;   // grid of the level (points per dim) and colour
    const double *b = nullptr; // EPI_STORE_DIAG: right-hand sides [M][ldb_diag]
    long ldb_diag = 0;
    double diag = 0.0;         // EPI_STORE_DIAG: first entry of the inverse column;
                               // EPI_RESID: coefficient of U (r_1 when acc is the history part)
    // EPI_RESID: the level's right-hand side F [M][P], iterate U (+ lo, its
    // double-double low part, or nullptr), c d_m, the initial condition g
    // (or nullptr) and 1/h^2; out has ldo = P
    const double *F = nullptr, *U = nullptr, *lo = nullptr, *cd = nullptr, *g = nullptr;
    double ih2 = 0.0;
    long ldu = 0;              // EPI_RESID*: row length of F, U, lo (the level's points)
    // EPI_RESID*: storage order (lay_pos) of F, U, lo (and of the product's
    // columns) and of out; EPI_RESID_R: of the coarse level written
    int lay_in = 0, lay_out = 0;
    // FP64 smoother products of a split level on the FFT route: the operand
    // is not stored but computed where the first pass reads it,
    // b = F + ih2 (neighbour sum) + cd g, from F (its first point the
    // colour's first, rows ldu apart) and the level's iterate U (the other
    // colour's values; rows ldu apart), g in natural order
    int rhs = 0;
    // FP64 residual on the FFT route (EPI_RESID, EPI_RESID_DD) in one chunk
    // of radix-256 passes: norm_part != nullptr: the last pass writes each
    // block's {max |r|, sum r^2} to norm_part[2 b], [2 b + 1]
    double *norm_part = nullptr;
};

// Tile choices of the product kernels (set by the autotuner).
struct TileKnobs {
    int variant = -1;          // wide FP64/FP32 kernel: 0 = 128x64, 1 = 256x64, -1 = by size
    int split_target = 0;      // work items a lone launch aims for (0 = default of the kernel)
};

struct GemmArgs {
    int mode = GM_F64;
    int M = 0;         // output rows (time levels)
    int P = 0;         // columns
    int K = 0;         // rows of B
    int off = 0;       // coefficient index s = off + i - k
    const ToepCoef *coef = nullptr;
    const void *B = nullptr;   // F64: double [K][ldb]; F32: float [K][ldb]
    const void *Bhi = nullptr; // BF16X3: uint16 k8-packed [Kpad/8][ldb][8]
    const void *Blo = nullptr;
    long ldb = 0;
    int epi = EPI_STORE;
    EpiArgs ea;
    void *part = nullptr;      // scratch for split-K partials
    size_t part_cap = 0;       // its size in bytes (0: never split)
    TileKnobs knobs;
    // FFT route (off = 0, K <= M): the causal product is the first M outputs
    // of a circular convolution of length fft_L >= 2M.  When fft_spec is set
    // the product runs as batched FFTs along time instead of the dense
    // kernels, in FP64 (mode GM_F64) or FP32 (other modes; spectra and
    // twiddles then FP32 complex, B FP64 if fft_b64 else FP32).
    const void *fft_spec = nullptr;  // complex [fft_L]: DFT of the coefficients, zero padded
    const void *fft_tw = nullptr;    // complex [fft_Ltw]: exp(-2 pi i k / fft_Ltw)
    int fft_L = 0, fft_Ltw = 0;      // powers of two, 64 <= fft_L <= fft_Ltw
    bool fft_b64 = true;
    // b_colour >= 0: product column j is point colour_point(ea.dims, ea.n,
    // b_colour, j) of B's rows (FFT route)
    int b_colour = -1;
    void *fft_buf0 = nullptr, *fft_buf1 = nullptr;  // work arrays, fft_buf_cap bytes each:
    size_t fft_buf_cap = 0;          // columns are transformed in chunks of 2 fft_buf_cap / (16 fft_L)
};

// Flat point index of the j-th point of a colour (0: n even / n + l even).
__host__ __device__ inline int colour_point(int dims, int n, int colour, int j)
{
    if (dims == 1) return colour == 0 ? 2 * j + 1 : 2 * j;
    int a = (colour == 0) ? (n + 1) / 2 : n / 2;   // points of the colour in an odd row
    int q = j / n, r = j - q * n;
    if (r < a) {   // row l = 2q + 1 (odd)
        int x = (colour == 0) ? 2 * r : 2 * r + 1;
        return (2 * q) * n + x;
    }
    r -= a;        // row l = 2q + 2 (even)
    int x = (colour == 0) ? 2 * r + 1 : 2 * r;
    return (2 * q + 1) * n + x;
}
__host__ __device__ inline int colour_count(int dims, int n, int colour)
{
    if (dims == 1) return colour == 0 ? n / 2 : (n + 1) / 2;
    long t = (long)n * n;
    return colour == 0 ? (int)((t + 1) / 2) : (int)(t / 2);
}

// Storage order of a level's points.  Natural (split == 0): x fastest.  Split
// by colour (split == 1): colour 0's points in the order of colour_point,
// then colour 1's, so that the points one half-sweep relaxes, and the
// neighbours its right-hand sides read, are contiguous.
// Storage index of the j-th point of colour c:
__host__ __device__ inline int lay_cpos(int dims, int n, int split, int c, int j)
{
    if (!split) return colour_point(dims, n, c, j);
    return (c == 0 ? 0 : colour_count(dims, n, 0)) + j;
}
// Storage index of natural point p (x + n y):
__host__ __device__ inline int lay_pos(int dims, int n, int split, int p)
{
    if (!split) return p;
    if (dims == 1) return (p & 1) ? (p >> 1) : (n >> 1) + (p >> 1);   // colour 0: odd p
    const int y = p / n, x = p - y * n, c = (x + y) & 1;
    // (as colour_point enumerates them) each pair of rows holds n points of
    // a colour; in the odd row of a pair they follow the (n + 1) / 2 (colour
    // 0) or n / 2 (colour 1) points of the even row, and in either row the
    // r-th point of the colour is at x = 2r or 2r + 1
    const int before = (y & 1) ? (c == 0 ? (n + 1) / 2 : n / 2) : 0;
    return (c == 0 ? 0 : colour_count(2, n, 0)) + (y >> 1) * n + before + (x >> 1);
}
// 2D forms that avoid divisions by n in the hot kernels: the j-th point of
// a colour as (x, y) (one division), the storage index of (x, y) (none) and
// the natural (x, y) of storage index s (one division).
__host__ __device__ inline void colour_xy(int n, int colour, int j, int &x, int &y)
{
    const int a = (colour == 0) ? (n + 1) / 2 : n / 2;
    const int q = j / n;
    int r = j - q * n;
    if (r < a) {
        y = 2 * q;
        x = (colour == 0) ? 2 * r : 2 * r + 1;
    } else {
        r -= a;
        y = 2 * q + 1;
        x = (colour == 0) ? 2 * r + 1 : 2 * r;
    }
}
__host__ __device__ inline int lay_pos_xy(int n, int split, int x, int y)
{
    if (!split) return y * n + x;
    const int c = (x + y) & 1;
    const int before = (y & 1) ? (c == 0 ? (n + 1) / 2 : n / 2) : 0;
    return (c == 0 ? 0 : (int)(((long)n * n + 1) / 2)) + (y >> 1) * n + before + (x >> 1);
}
__host__ __device__ inline void lay_xy(int n, int split, int s, int &x, int &y)
{
    if (!split) {
        y = s / n;
        x = s - y * n;
        return;
    }
    const int p0 = (int)(((long)n * n + 1) / 2);
    if (s < p0) colour_xy(n, 0, s, x, y);
    else colour_xy(n, 1, s - p0, x, y);
}
// Natural point of storage index s:
__host__ __device__ inline int lay_nat(int dims, int n, int split, int s)
{
    if (!split) return s;
    const int p0 = colour_count(dims, n, 0);
    return s < p0 ? colour_point(dims, n, 0, s) : colour_point(dims, n, 1, s - p0);
}

// ---------------------------------------------------------------------------
// Argument arrays of grouped launches.  A stage is run twice over the same
// host logic: a RECORD pass appends every array to `host` and launches
// nothing; after `dev` holds a copy of `host`, the LAUNCH pass makes the same
// calls, gets the same offsets back as device addresses, and launches.
struct Staging {
    bool record = false;
    std::vector<char> host;
    char *dev = nullptr;
    size_t cursor = 0;
    const void *put(const void *p, size_t bytes)
    {
        size_t at = (cursor + 255) & ~(size_t)255;
        cursor = at + bytes;
        if (record) {
            host.resize(cursor);
            memcpy(host.data() + at, p, bytes);
            return nullptr;
        }
        return dev + at;
    }
};

// ---- argument sets of the bandwidth kernels ----
// Colour right-hand side b = F + cd g + (neighbour sum of U)/h^2 at the
// points of a colour, as the B operand of the smoother's product: fmt 0:
// FP64 panel [M][ldp]; 1: FP32 panel [M][ldp]; 2: split-BF16 k8-packed
// [Mpad/8][ldp][8] (hi into panel, lo into panel_lo; zero for k >= M, j >= Pc).
// If lam0 != 0 the kernel also writes lam0 * b into the colour's points of U
// (the diagonal part of the line solve; the product then adds the history).
struct RhsArgs {
    int fmt, dims, n, colour, M, Mpad;
    const double *F;
    double *U;
    const double *cd, *g;
    double ih2, lam0;
    void *panel, *panel_lo;
    long ldp;
    int split = 0;          // storage order of F and U (lay_pos)
    int zero_nbrs = 0;      // the iterate is zero: no neighbour values are read (b = F + c d g)
};
// Residual from a Toeplitz product already in out (the history part, or all
// of T_M U when diag = 0): out = (F + cd g - diag U - A_h U) - out, with A_h
// applied to U + lo by error-free transformations when lo != nullptr.
struct PostArgs {
    int dims, n, M;
    const double *F, *U, *lo, *cd, *g;
    double ih2, diag;
    double *out;
    int lay_in = 0, lay_out = 0;     // storage order of F, U, lo, prod and of out
    const double *prod = nullptr;    // the product (nullptr: in out, lay_in == lay_out)
};
// Low-precision product operand of rows [0, M) of X [.][ldx] (P columns):
// fmt 1: FP32 [M][ldp]; fmt 2: split-BF16 k8-packed [Mpad/8][ldp][8] (rows
// M..Mpad-1 and columns P..ldp-1 zero).  If X2 != nullptr it also writes
// X2 = s2 * X ([.][ldx]; the D&C base block's diagonal part).
struct OperandArgs {
    int fmt, M, Mpad, P;
    const double *X;
    long ldx;
    void *out, *out_lo;
    long ldp;
    double *X2;
    double s2;
};
// Full weighting (dir 0: fine n -> coarse) or interpolation added to the
// fine iterate (dir 1: coarse n -> fine).
struct XferArgs {
    int dir, dims, n, M;
    const double *src;
    double *dst;
    int zero_colour = -1;   // restriction: src holds only the other colour (this one is zero)
    int split = 0;          // storage order of both levels
    // restriction: the residual is not stored but implied by the iterate src
    // of a level that started from zero and was smoothed by one red-black
    // sweep (first colour = 1 - zero_colour): ih2 times the neighbour sum of
    // src at the first colour's points, zero at the others
    int implicit = 0;
    double ih2 = 0.0;
    // interpolation: this colour's fine points are not corrected (the first
    // half-sweep of the post-smoothing recomputes them from the other
    // colour alone); -1: all points
    int skip_colour = -1;
};
// u[k][s] = scaled ? cd[k] g[p] : g[p] for the natural point p of storage
// index s (g == nullptr: 0)
struct FillArgs {
    long M, P;
    const double *cd, *g;
    double *u;
    int scaled;
    int dims = 1, n = 0, split = 0;   // storage order of u (split: dims and n give it)
};
// Norm partials {max |x|, sum x^2} of x[0..n) over nblk blocks, and the final
// reduction into out2 = {max, sqrt(sum)}.
struct NormArgs {
    long n;
    const double *x;
    double *partials;
    int nblk;
    double *out2;
    int have_partials = 0;   // the partials were written by the product (only the final reduction)
};
// (hi, lo) += e (double-double); lo == nullptr: hi += e.  hi and lo in
// natural order; e in the storage order `split` of a level with npd points
// per dimension (n = M x points values).
struct DDArgs {
    long n;
    const double *e;
    double *hi, *lo;
    int dims = 1, npd = 0, split = 0;
};
// U[k][colour's j-th point] = X[k][j], k < M, j < Pc (end of a D&C half-sweep).
struct ScatterArgs {
    int dims, n, colour, M, Pc;
    const double *X;
    double *U;
    int split = 0;
};
// Reorder [M][points] between natural order and the split storage order:
// to_split: dst[k][lay_pos(p)] = src[k][p]; else dst[k][p] = src[k][lay_pos(p)].
struct PermuteArgs {
    int dims, n, M, to_split;
    const double *src;
    double *dst;
};

// ---- launchers (all asynchronous on `s`; st may be nullptr when every list
// has at most one entry) ----
hipError_t launch_toep_gemm(const std::vector<GemmArgs> &as, Staging *st, hipStream_t s);
// Scratch a lone product of this shape uses for split-K partials (0: not split).
size_t splitk_bytes(int mode, int M, int P, int K, int off, int ncoef, const TileKnobs &kn);
hipError_t launch_rhs(const std::vector<RhsArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_post(const std::vector<PostArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_operand(const std::vector<OperandArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_xfer(const std::vector<XferArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_fill(const std::vector<FillArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_norms(const std::vector<NormArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_dd_update(const std::vector<DDArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_scatter(const std::vector<ScatterArgs> &v, Staging *st, hipStream_t s);
hipError_t launch_permute(const std::vector<PermuteArgs> &v, Staging *st, hipStream_t s);
// Bytes the FFT route's passes move through their complex work arrays for
// one product (written by the first kernel, read and written by each middle
// one, read by the last).
double fft_work_bytes(const GemmArgs &a);
// Whether an FFT-route product runs as one on-chip kernel (FP64, L <= 4096,
// plain input, store or scatter epilogue).
bool fft_on_chip(const GemmArgs &a);
// Blocks of the last pass of an FP64 FFT-route product whose columns fit its
// work arrays in one chunk and whose transform uses the radix-256 passes
// (the residual products that can write norm partials); 0 for any other.
long fft_fused_blocks(const GemmArgs &a);
// Fill one coefficient table (fp32 copy and bf16 fragment table) from d64.
hipError_t launch_build_coef(ToepCoef &c, hipStream_t s);
// Blocks of the norm partials of an n-element array.
int norm_partial_blocks(long n);
// Device address of this device's static scratch (MGWR_STATIC_SCRATCH_BYTES
// bytes); `device` must be current.  Looked up once per device.
int static_scratch(int device, void **ptr);

}  // namespace mgwr
