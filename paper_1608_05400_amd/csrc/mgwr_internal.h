// Internal interfaces of the MGWR library: device data layouts and the
// kernel launchers the host runtime (mgwr_capi.cpp) drives.
//
// All grid functions (iterates, right-hand sides, residuals) are FP64 in HBM,
// time-major [M][P].  Only the operands of the Toeplitz products may be held
// in lower precision (FP32 panels, or split-BF16 hi/lo panels in the k8-packed
// layout [Mpad/8][ld][8]).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mgwr {

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
enum EpiKind {
    EPI_STORE = 0,       // out[i][p] = acc                        (residual product)
    EPI_SCATTER = 1,     // out[i][colour_point(p)] = acc          (smoother, full product)
    EPI_SCATTER_ADD = 2, // out[i][colour_point(p)] += acc         (smoother, history product)
    EPI_SUB = 3          // out[i][p] -= acc                       (D&C history update)
};

struct EpiArgs {
    double *out = nullptr;     // output (STORE/SUB) or the iterate U of the level (SCATTER*)
    long ldo = 0;
    int dims = 1, n = 1, colour = 0;   // grid of the level (points per dim) and colour
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

// ---- launchers (all asynchronous on `s`) ----
hipError_t launch_toep_gemm(const GemmArgs &a, hipStream_t s);
// Scratch a product of this shape uses for split-K partials (0: not split).
size_t splitk_bytes(int mode, int M, int P, int K, int off, int ncoef);

// Right-hand side of a colour half-sweep, b = F + cd g + (neighbour sum of U)/h^2
// at the points of the colour, as the B operand of the smoother's product:
// fmt 0: FP64 panel [M][ldp]; 1: FP32 panel [M][ldp]; 2: split-BF16 k8-packed
// [Mpad/8][ldp][8] (hi into panel, lo into panel_lo; zero for k >= M, j >= Pc).
// If lam0 != 0 the kernel also writes lam0 * b into the colour's points of U
// (the diagonal part of the line solve; the product then adds the history).
hipError_t launch_rhs_panel(int fmt, int dims, int n, int colour, int M, int Mpad, const double *F,
                            double *U, const double *cd, const double *g, double ih2, double lam0,
                            void *panel, void *panel_lo, long ldp, hipStream_t s);
// Residual from a Toeplitz product already in out (the history part, or all of
// T_M U when diag = 0): out = (F + cd g - diag U - A_h U) - out, with A_h
// applied to hi + lo by error-free transformations when lo != nullptr.
hipError_t launch_resid_post(int dims, int n, int M, const double *F, const double *U, const double *lo,
                             const double *cd, const double *g, double ih2, double diag, double *out,
                             hipStream_t s);
// X [M][P] FP64 -> FP32 copy [M][P] (fmt 1) or split-BF16 k8-packed (fmt 2).
hipError_t launch_operand(int fmt, int M, int Mpad, int P, const double *X, void *out,
                          void *out_lo, long ldp, hipStream_t s);
hipError_t launch_restrict(int dims, int nf, int M, const double *rf, double *rc, hipStream_t s);
hipError_t launch_prolong_add(int dims, int nc, int M, const double *ec, double *uf, hipStream_t s);
// u[k][p] = g ? g[p] : 0
hipError_t launch_fill(long M, long P, const double *g, double *u, hipStream_t s);
// u[k][p] = g ? cd[k] g[p] : 0
hipError_t launch_scaled_fill(long M, long P, const double *cd, const double *g, double *u, hipStream_t s);
// Block partials of {max |x|, sum x^2}; partials: [nblk][2]; returns nblk.
hipError_t launch_norm_partials(long n, const double *x, double *partials, int *nblk,
                                hipStream_t s);
hipError_t launch_norm_final(int nblk, const double *partials, double *out2, hipStream_t s);
// (hi, lo) += e (double-double); lo == nullptr: hi += e.
hipError_t launch_dd_update(long n, const double *e, double *hi, double *lo, hipStream_t s);
// FP32 -> FP64 copy.
hipError_t launch_widen(long n, const float *x, double *y, hipStream_t s);
// Fill one coefficient table (fp32 copy and bf16 fragment table) from d64.
hipError_t launch_build_coef(ToepCoef &c, hipStream_t s);
int norm_partial_blocks(long n);

}  // namespace mgwr
