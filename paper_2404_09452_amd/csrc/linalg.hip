// Dense FP64 linear algebra on the auxiliary metric, gfx950:
//   - blocked right-looking Cholesky V = L L^T (64-wide panels; the diagonal
//     block is factored in registers by one wave, which also inverts it; the
//     panel below is multiplied by that inverse and the trailing matrix
//     updated, both on FP64 MFMA),
//   - L^{-1} by blocked forward substitution on the identity, block row by
//     block row (row i needs only the factor steps up to i),
//   - the whitening B = U L^{-T}-transposed product, i.e. B[f][P] =
//     sum_{Q<=P} U[f][Q] Linv[P][Q], as one MFMA GEMM that stops each output
//     tile's k loop at its last column (Linv is lower triangular).
// Matrices are row-major with the padded leading dimension npad (a multiple
// of 64); the pad block of the metric is the identity so every factor stays
// well defined and the pad rows/columns of B are exactly zero.
#include <climits>

#include "dfjk_internal.h"
#include "gemm_f64.h"

namespace dfjk {

constexpr int NBK = 64;   // panel width

__global__ void k_metric_pad(double *V, int64_t n, int64_t npad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad * npad) return;
    const int64_t r = i / npad, c = i % npad;
    if (r >= n || c >= n) V[i] = (r == c) ? 1.0 : 0.0;
}

void launch_metric_pad(double *V, int64_t n, int64_t npad, hipStream_t s)
{
    const int64_t tot = npad * npad;
    hipLaunchKernelGGL(k_metric_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, n, npad);
}

// Lane `src`'s value of v, broadcast to the wave (two 32-bit lane reads).
__device__ __forceinline__ double readlane_f64(double v, int src)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, src);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Factor the 64x64 diagonal block at (k0, k0) in place with one wave: lane i
// holds row i in registers.  Step j takes the pivot from lane j by a lane
// read, scales column j, publishes the column through LDS (one wave, so a
// barrier per step orders the write before the broadcast reads) and updates
// every later column of every row with one FMA per entry.  Entries above the
// diagonal are updated too but never read by a later step (a step reads the
// pivot from its own lane and the column from the rows below it) and are
// stored as zero.  A pivot <= 0 is recorded (smallest index wins) and
// replaced by 1 so the remaining steps stay finite; the host reports the
// recorded index.
__global__ __launch_bounds__(64) void k_potrf_diag(double *A, int64_t ld, int64_t k0, int32_t *status, double *Dk)
{
    __shared__ __align__(16) double col[2][NBK];
    constexpr int LDT = NBK + 2;
    __shared__ __align__(16) double LT[NBK * LDT];
    const int i = threadIdx.x;
    double *row = A + (k0 + i) * ld + k0;
    double r[NBK];
#pragma unroll
    for (int c = 0; c < NBK; ++c) r[c] = row[c];
    int bad = INT_MAX;
#pragma unroll
    for (int j = 0; j < NBK; ++j) {
        double d = readlane_f64(r[j], j);
        if (!(d > 0.0)) {
            if (bad == INT_MAX) bad = (int)(k0 + j);
            d = 1.0;
        }
        d = sqrt(d);
        r[j] = (i == j) ? d : r[j] / d;
        double *cj = col[j & 1];
        cj[i] = r[j];
        __syncthreads();
        // L[l][j] for l > j: an odd first entry alone, then 16-byte aligned pairs
        int l0 = j + 1;
        if ((l0 & 1) && l0 < NBK) {
            r[l0] = fma(-r[j], cj[l0], r[l0]);
            ++l0;
        }
#pragma unroll
        for (int l = l0; l < NBK; l += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(cj + l);
            r[l] = fma(-r[j], v.x, r[l]);
            r[l + 1] = fma(-r[j], v.y, r[l + 1]);
        }
    }
    if (i == 0 && bad != INT_MAX) atomicMin(status, bad);
#pragma unroll
    for (int c = 0; c < NBK; ++c) {
        const double v = (c <= i) ? r[c] : 0.0;
        row[c] = v;
        LT[c * LDT + i] = v;          // L_kk transposed: row l holds column l
    }
    __syncthreads();
    // Dk = L_kk^{-1}: column t by forward substitution of e_t, right-looking:
    // x_l is final once divided by L_ll, and its column of L (a row of LT,
    // 16-byte aligned) updates every later entry with independent FMAs
    const int t = i;
    double x[NBK];
#pragma unroll
    for (int q = 0; q < NBK; ++q) x[q] = (q == t) ? 1.0 : 0.0;
#pragma unroll
    for (int l = 0; l < NBK; ++l) {
        const double *cl = LT + l * LDT;
        x[l] = x[l] / cl[l];
        int q0 = l + 1;
        if ((q0 & 1) && q0 < NBK) {
            x[q0] = fma(-cl[q0], x[l], x[q0]);
            ++q0;
        }
#pragma unroll
        for (int q = q0; q < NBK; q += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(cl + q);
            x[q] = fma(-v.x, x[l], x[q]);
            x[q + 1] = fma(-v.y, x[l], x[q + 1]);
        }
    }
#pragma unroll
    for (int q = 0; q < NBK; ++q) Dk[q * NBK + t] = x[q];
}

// Step k of the blocked Cholesky: factor and invert the diagonal block,
// form the panel below it, update the trailing matrix.
void cholesky_step(double *A, int64_t npad, int64_t k, int32_t *status, double *Dinv, hipStream_t s)
{
    const int64_t nb = npad / NBK;
    const int64_t k0 = k * NBK;
    double *Dk = Dinv + k * NBK * NBK;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(NBK), 0, s, A, npad, k0, status, Dk);
    const int64_t rest = nb - k - 1;
    if (rest == 0) return;
    // panel: L21 = A21 L_kk^{-T} = A21 Dk^T on MFMA, in place (each output
    // tile reads only its own 64 rows, wholly, before writing them)
    GemmArgs pg{};
    pg.A = A + (k0 + NBK) * npad + k0; pg.lda = npad;
    pg.B = Dk; pg.ldb = NBK;
    pg.C = A + (k0 + NBK) * npad + k0; pg.ldc = npad;
    pg.M = rest * NBK; pg.N = NBK;
    pg.k_begin = 0; pg.k_end = NBK; pg.ksplit = NBK;
    pg.alpha = 1.0; pg.beta = 0.0;
    gemm_f64<64, false>(pg, 1, s);
    // A22 -= L21 L21^T on the lower tiles of the trailing matrix
    GemmArgs g{};
    const int64_t t0 = k0 + NBK;
    g.A = A + t0 * npad + k0; g.lda = npad;
    g.B = A + t0 * npad + k0; g.ldb = npad;
    g.C = A + t0 * npad + t0; g.ldc = npad;
    g.M = g.N = npad - t0;
    g.k_begin = 0; g.k_end = NBK; g.ksplit = NBK;
    g.alpha = -1.0; g.beta = 1.0; g.lower = 1;
    gemm_f64<64, false>(g, 1, s);
}

void launch_cholesky(double *A, int64_t npad, int32_t *status, double *Dinv, hipStream_t s)
{
    for (int64_t k = 0; k < npad / NBK; ++k) cholesky_step(A, npad, k, status, Dinv, s);
}

__global__ void k_zero_upper(double *A, int64_t npad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad * npad) return;
    if (i % npad > i / npad) A[i] = 0.0;
}

__global__ void k_identity(double *A, int64_t npad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad * npad) return;
    A[i] = (i % npad == i / npad) ? 1.0 : 0.0;
}

void launch_zero_upper(double *L, int64_t npad, hipStream_t s)
{
    const int64_t tot = npad * npad;
    hipLaunchKernelGGL(k_zero_upper, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L, npad);
}

void trtri_begin(double *X, int64_t npad, hipStream_t s)
{
    const int64_t tot = npad * npad;
    hipLaunchKernelGGL(k_identity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, npad);
}

// X = L^{-1} by blocked forward substitution on the identity, block row i at
// a time: X_i[0:w] <- D_i X_i[0:w] (w = (i+1) 64, D_i = L_ii^{-1} from the
// factor's diagonal step; an MFMA GEMM, in place: each output tile reads only
// its own 64 x 64 block of X_i, wholly, before writing it), then
// X[rows below][0:w] -= L[rows below][block i] X_i[0:w].  Step i reads only
// what Cholesky steps 0..i have finished (D_i and the strictly lower column
// block i of L), so it can follow step i on another stream.
void trtri_step(const double *L, double *X, const double *Dinv, int64_t npad, int64_t i, hipStream_t s)
{
    const int64_t nb = npad / NBK;
    const int64_t i0 = i * NBK, w = i0 + NBK;
    GemmArgs d{};
    d.A = Dinv + i * NBK * NBK; d.lda = NBK;
    d.B = X + i0 * npad; d.ldb = npad;
    d.C = X + i0 * npad; d.ldc = npad;
    d.M = NBK; d.N = w;
    d.k_begin = 0; d.k_end = NBK; d.ksplit = NBK;
    d.alpha = 1.0; d.beta = 0.0;
    gemm_f64<64, true>(d, 1, s);
    if (i + 1 == nb) return;
    // X[j rows > i][0:w] -= L[j rows][i cols] X[i rows][0:w]
    GemmArgs g{};
    g.A = L + w * npad + i0; g.lda = npad;
    g.B = X + i0 * npad; g.ldb = npad;
    g.C = X + w * npad; g.ldc = npad;
    g.M = npad - w; g.N = w;
    g.k_begin = 0; g.k_end = NBK; g.ksplit = NBK;
    g.alpha = -1.0; g.beta = 1.0;
    gemm_f64<64, true>(g, 1, s);
}

// L^{-1} after the whole factor (Dinv as launch_cholesky left it); the upper
// triangle of L is zeroed for the callers that read L itself.
void launch_trtri(double *L, double *X, const double *Dinv, int64_t npad, hipStream_t s)
{
    launch_zero_upper(L, npad, s);
    trtri_begin(X, npad, s);
    for (int64_t i = 0; i < npad / NBK; ++i) trtri_step(L, X, Dinv, npad, i, s);
}

void launch_whiten(const double *U, const double *Linv, double *B, int64_t nf_pad, int64_t npad, hipStream_t s)
{
    launch_gemm_nt_tri(U, Linv, B, nf_pad, npad, npad, s);
}

}  // namespace dfjk
