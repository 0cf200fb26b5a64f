// Orbital alignment for the incremental build (dfjk_build_delta).  D = C C^T
// does not change under C -> C Q for any orthogonal Q (a sign flip or a
// rotation of the occupied orbitals among themselves), but the increment's
// operand W = C - C0 does: the mixed-precision error of K(D) = K0 + G + G^T,
// G = X_{C+C0} X_{C-C0}^T, scales with |W|.  So C is first rotated onto C0:
// Q is the orthogonal polar factor of M = C^T C0, the minimiser of
// |C Q - C0|_F (orthogonal Procrustes problem; Schoenemann, Psychometrika 31,
// 1966), by the Newton-Schulz iteration X <- X (3 I - X^T X) / 2 from
// X0 = M / |M|_F, which converges to the polar factor when every singular
// value of X0 lies in (0, sqrt 3) (Higham, Functions of Matrices, Ch. 8).
// A fixed count of iterations keeps the build free of host synchronisation;
// if X^T X then differs from I by more than 1e-13 anywhere (M near singular:
// C and C0 span different spaces), Q = I and C is used as given.
#include "dfjk_internal.h"

namespace dfjk {

constexpr int kAlignIters = 40;
constexpr double kAlignTol = 1e-13;

// C = alpha op(A) op(B) + beta C, small dense FP64 (32 x 32 tiles, LDS)
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_small(int M, int N, int K, const double *__restrict__ A, int lda,
                                                    const double *__restrict__ B, int ldb, double *__restrict__ C,
                                                    int ldc, double alpha, double beta)
{
    __shared__ double As[32][33], Bs[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;      // 32 x 8 threads, 4 rows each
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 32) {
        for (int q = threadIdx.x; q < 32 * 32; q += 256) {
            const int r = q / 32, c = q % 32;                        // r: m (or k), c: k (or n)
            const int m = m0 + r, ka = k0 + c;
            As[r][c] = (m < M && ka < K) ? (TA ? A[(int64_t)ka * lda + m] : A[(int64_t)m * lda + ka]) : 0.0;
            const int kb = k0 + r, n = n0 + c;
            Bs[r][c] = (kb < K && n < N) ? (TB ? B[(int64_t)n * ldb + kb] : B[(int64_t)kb * ldb + n]) : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < 32; ++k) {
            const double b = Bs[k][tx];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] = fma(As[ty + 8 * i][k], b, acc[i]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty + 8 * i, n = n0 + tx;
        if (m < M && n < N) {
            double *c = C + (int64_t)m * ldc + n;
            *c = alpha * acc[i] + (beta == 0.0 ? 0.0 : beta * *c);
        }
    }
}

// stat[0] = sqrt(sum M^2) (one block)
__global__ __launch_bounds__(256) void k_frob(const double *__restrict__ M, int64_t n, double *__restrict__ stat)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += M[e] * M[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) stat[0] = sqrt(red[0]);
}

// X = M / stat[0] (X = I when M is zero)
__global__ void k_scale_start(const double *__restrict__ M, int nocc, const double *__restrict__ stat,
                              double *__restrict__ X)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nocc * nocc) return;
    const double f = stat[0];
    X[e] = f > 0.0 ? M[e] / f : ((e / nocc == e % nocc) ? 1.0 : 0.0);
}

// T = (3 I - Y) / 2
__global__ void k_ns_t(const double *__restrict__ Y, int nocc, double *__restrict__ T)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nocc * nocc) return;
    T[e] = ((e / nocc == e % nocc) ? 1.5 : 0.0) - 0.5 * Y[e];
}

// Q = X when max |Y - I| <= tol (Y = X^T X), else Q = I (one block)
__global__ __launch_bounds__(256) void k_orth_check(const double *__restrict__ X, const double *__restrict__ Y,
                                                    int nocc, double *__restrict__ Q, double tol)
{
    __shared__ double red[256];
    const int64_t n = (int64_t)nocc * nocc;
    double d = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) {
        const double v = fabs(Y[e] - ((e / nocc == e % nocc) ? 1.0 : 0.0));
        d = (v > d || v != v) ? v : d;        // NaN counts as failure
    }
    red[threadIdx.x] = d;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    const bool ok = red[0] <= tol;
    for (int64_t e = threadIdx.x; e < n; e += 256) Q[e] = ok ? X[e] : ((e / nocc == e % nocc) ? 1.0 : 0.0);
}

size_t align_work_doubles(int32_t nocc) { return (size_t)5 * nocc * nocc + 64; }

// Cr = C Q with Q the orthogonal polar factor of C^T C0 (or I, see above).
// work: align_work_doubles(nocc) doubles.
void launch_align(const double *C, const double *C0, int64_t nao, int32_t nocc, double *work, double *Cr,
                  hipStream_t s)
{
    const int n = nocc;
    const int64_t nn = (int64_t)n * n;
    double *M = work, *X = M + nn, *X2 = X + nn, *Y = X2 + nn, *T = Y + nn, *stat = T + nn;
    const dim3 g_small((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
    const unsigned g_elem = (unsigned)((nn + 255) / 256);
    // M = C^T C0 (nocc x nocc over nao)
    hipLaunchKernelGGL((k_gemm_small<true, false>), g_small, dim3(256), 0, s, n, n, (int)nao, C, n, C0, n, M, n,
                       1.0, 0.0);
    hipLaunchKernelGGL(k_frob, dim3(1), dim3(256), 0, s, M, nn, stat);
    hipLaunchKernelGGL(k_scale_start, dim3(g_elem), dim3(256), 0, s, M, n, stat, X);
    for (int it = 0; it < kAlignIters; ++it) {
        hipLaunchKernelGGL((k_gemm_small<true, false>), g_small, dim3(256), 0, s, n, n, n, X, n, X, n, Y, n, 1.0,
                           0.0);
        hipLaunchKernelGGL(k_ns_t, dim3(g_elem), dim3(256), 0, s, Y, n, T);
        hipLaunchKernelGGL((k_gemm_small<false, false>), g_small, dim3(256), 0, s, n, n, n, X, n, T, n, X2, n, 1.0,
                           0.0);
        double *t = X;
        X = X2;
        X2 = t;
    }
    hipLaunchKernelGGL((k_gemm_small<true, false>), g_small, dim3(256), 0, s, n, n, n, X, n, X, n, Y, n, 1.0, 0.0);
    hipLaunchKernelGGL(k_orth_check, dim3(1), dim3(256), 0, s, X, Y, n, T, kAlignTol);
    // Cr = C Q (nao x nocc)
    const dim3 g_c((unsigned)((n + 31) / 32), (unsigned)((nao + 31) / 32));
    hipLaunchKernelGGL((k_gemm_small<false, false>), g_c, dim3(256), 0, s, (int)nao, n, n, C, n, T, n, Cr, n, 1.0,
                       0.0);
}

}  // namespace dfjk

namespace dfjk {

// stat[s] = |P|_F for the s-th squaring's product, then P /= stat[s]
__global__ __launch_bounds__(256) void k_frob_scale(double *__restrict__ P, int64_t n, double *__restrict__ stat)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += P[e] * P[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double f = sqrt(red[0]);
    __syncthreads();
    if (threadIdx.x == 0) stat[0] = f;
    if (f > 0.0)
        for (int64_t e = threadIdx.x; e < n; e += 256) P[e] /= f;
}

// out[0] = |M|_F, out[1] >= lambda_max(M), M = C^T C: |M^16|_F^(1/16) =
// f_0 g_1^(1/2) g_2^(1/4) g_3^(1/8) g_4^(1/16) with f_0 = |M|_F and g_t the
// norm of the t-th normalised square (the Frobenius norm bounds the spectral
// one, and |M^16|_2 = lambda_max^16), times 1 + 1e-12 for the rounding of
// the products.
__global__ void k_gram_bound(const double *__restrict__ stat, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = stat[0];
    for (int t = 1; t <= kGramSquarings; ++t) l *= pow(stat[t], 1.0 / (double)(1 << t));
    out[0] = stat[0];
    out[1] = l * (1.0 + 1e-12);
}

size_t gram_work_doubles(int32_t nocc) { return (size_t)2 * nocc * nocc + 16; }

void launch_gram_bound(const double *C, int64_t nao, int32_t nocc, double *work, double *out, hipStream_t s)
{
    const int n = nocc;
    const int64_t nn = (int64_t)n * n;
    double *P = work, *P2 = P + nn, *stat = P2 + nn;
    const dim3 g_small((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
    hipLaunchKernelGGL((k_gemm_small<true, false>), g_small, dim3(256), 0, s, n, n, (int)nao, C, n, C, n, P, n,
                       1.0, 0.0);
    hipLaunchKernelGGL(k_frob_scale, dim3(1), dim3(256), 0, s, P, nn, stat);
    for (int t = 1; t <= kGramSquarings; ++t) {
        hipLaunchKernelGGL((k_gemm_small<false, false>), g_small, dim3(256), 0, s, n, n, n, P, n, P, n, P2, n, 1.0,
                           0.0);
        hipLaunchKernelGGL(k_frob_scale, dim3(1), dim3(256), 0, s, P2, nn, stat + t);
        double *tmp = P;
        P = P2;
        P2 = tmp;
    }
    hipLaunchKernelGGL(k_gram_bound, dim3(1), dim3(64), 0, s, stat, out);
}

}  // namespace dfjk
