// Rigorous bound on the energy error of the int8 K build, from the stored
// slices of X (dfjk_build_checked).
//
// With x = x~ + r per element (x~ the five-slice reconstruction
// sum_s alpha_s, alpha_s = a_s 2^{e - 7(s+1)}, |r| <= 2^{e-36}), the int8
// product of x_mu and x_nu is x~_mu x~_nu minus the dropped orders
// t = sum_{i+j>=5} alpha_i alpha_j.  For the closed-shell energy
// E_K = -1/2 sum_k x_k^T D x_k (K = 2 X X^T, D = 2 C C^T), the difference
// between the int8 energy and the same X contracted exactly is
//   1/2 sum_k [2 x~_k^T D r_k + r_k^T D r_k + sum_{i+j>=5} alpha_ik^T D alpha_jk].
// D is positive semidefinite, so |u^T D v| <= sqrt(u^T D u) sqrt(v^T D v)
// (Cauchy-Schwarz in the D-seminorm, then over k), and u^T D u <=
// lambda |u|^2 with lambda >= lambda_max(D) = 2 lambda_max(C^T C):
//   |dE_K| <= 1/2 [2 sqrt(Q lambda R) + lambda R + lambda T] + F,
//   A_s = sum_k |alpha_sk|^2 (exact, from the digits),
//   R = sum over blocks of 256 2^{2e - 72} >= sum_k |r_k|^2,
//   T = sum_{i+j>=5, 1<=i,j<=4} sqrt(A_i A_j),
//   Q = 2 |E_K(int8)| + lambda T + 2F >= sum_k x~_k^T D x~_k,
//   F = gamma_n |D|_F (sum_s sqrt A_s)^2, gamma_n = n u / (1 - n u), u = 2^-53,
// F covering the FP64 rounding of the block folds and of the split and slab
// sums (n of them per element).  This is the Section 5 idea of the paper
// (estimate the error of the lower-precision part and keep it below what the
// result needs) made rigorous for this format.
#include "dfjk_internal.h"

namespace dfjk {

// acc[mu][s] += A_s of row mu (s < 5), acc[mu][5] += the R term of row mu,
// for one slab's int8 X ([nao][kdim/64][5][64] bytes) and its block scales
// ([nao][kdim/256]).  One workgroup per row; each thread sums whole 16-byte
// pieces (16 consecutive k of one slice) in a fixed order, then a fixed-order
// tree: the sums are deterministic.
__global__ __launch_bounds__(256) void k_i8_norms(const unsigned char *__restrict__ X,
                                                  const double *__restrict__ scales, int64_t kdim,
                                                  double *__restrict__ acc)
{
    const int64_t mu = blockIdx.x;
    const int64_t nblk = kdim / kI8Block;
    const unsigned char *row = X + mu * kdim * kI8Slices;
    const double *sc = scales + mu * nblk;
    constexpr int kUnitsPerBlock = (kI8Block / kI8Chunk) * kI8Slices * (kI8Chunk / 16);   // 80
    double s[kI8Slices + 1] = {};
    for (int64_t u = threadIdx.x; u < nblk * kUnitsPerBlock; u += 256) {
        const int64_t b = u / kUnitsPerBlock;
        const int r = (int)(u % kUnitsPerBlock);
        const int chunk = r / (kI8Slices * 4), sl = (r / 4) % kI8Slices, q = r % 4;
        const int64_t off = ((b * (kI8Block / kI8Chunk) + chunk) * kI8Slices + sl) * kI8Chunk + q * 16;
        const uint4 v = *reinterpret_cast<const uint4 *>(row + off);
        const unsigned int w[4] = {v.x, v.y, v.z, v.w};
        int sq = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int a = (int)(signed char)(w[i] >> (8 * j));
                sq += a * a;
            }
        const double f = sc[b];
        // (a 2^{e - 7(s+1)})^2 = a^2 (2^e)^2 2^{-14(s+1)}
#pragma unroll
        for (int t = 0; t < kI8Slices; ++t)
            if (t == sl) s[t] += ldexp((double)sq * f * f, -14 * (t + 1));
    }
    for (int64_t b = threadIdx.x; b < nblk; b += 256) s[kI8Slices] += ldexp(256.0 * sc[b] * sc[b], -72);
    __shared__ double red[kI8Slices + 1][256];
#pragma unroll
    for (int t = 0; t <= kI8Slices; ++t) red[t][threadIdx.x] = s[t];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int t = 0; t <= kI8Slices; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x <= kI8Slices) acc[mu * (kI8Slices + 1) + threadIdx.x] += red[threadIdx.x][0];
}

// out[0] = the bound (Eh); out[1..4] = lambda, Q, R, T (diagnostics).
// gram: {|C^T C|_F, upper bound of lambda_max(C^T C)}; E[1] the int8 E_K.
__global__ __launch_bounds__(256) void k_i8_bound(const double *__restrict__ acc, int64_t nao,
                                                  const double *__restrict__ gram, const double *__restrict__ E,
                                                  int nsums, double *__restrict__ out)
{
    __shared__ double red[kI8Slices + 1][256];
    double s[kI8Slices + 1] = {};
    for (int64_t mu = threadIdx.x; mu < nao; mu += 256)
#pragma unroll
        for (int t = 0; t <= kI8Slices; ++t) s[t] += acc[mu * (kI8Slices + 1) + t];
#pragma unroll
    for (int t = 0; t <= kI8Slices; ++t) red[t][threadIdx.x] = s[t];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int t = 0; t <= kI8Slices; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double As[kI8Slices];
    for (int t = 0; t < kI8Slices; ++t) As[t] = red[t][0];
    const double R = red[kI8Slices][0];
    double T = 0.0;
    for (int i = 1; i < kI8Slices; ++i)
        for (int j = 1; j < kI8Slices; ++j)
            if (i + j >= kI8Slices) T += sqrt(As[i] * As[j]);
    const double lam = 2.0 * gram[1];
    const double dF = 2.0 * gram[0];                 // |D|_F = 2 |C C^T|_F = 2 |C^T C|_F
    double xs = 0.0;
    for (int t = 0; t < kI8Slices; ++t) xs += sqrt(As[t]);
    const double n = (double)nsums, u = 0x1p-53;
    const double F = n * u / (1.0 - n * u) * dF * xs * xs;
    const double Q = 2.0 * fabs(E[1]) + lam * T + 2.0 * F;
    const double bound = 0.5 * (2.0 * sqrt(Q * lam * R) + lam * R + lam * T) + F;
    out[0] = bound * (1.0 + 1e-12);
    out[1] = lam;
    out[2] = Q;
    out[3] = R;
    out[4] = T;
}

size_t i8_bound_work_doubles(int64_t nao, int32_t nocc)
{
    return (size_t)nao * (kI8Slices + 1) + gram_work_doubles(nocc) + 16;
}

void launch_i8_norms(const void *X, const double *scales, int64_t nao, int64_t kdim, double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_i8_norms, dim3((unsigned)nao), dim3(256), 0, s, static_cast<const unsigned char *>(X),
                       scales, kdim, acc);
}

void launch_i8_bound(const double *C, int64_t nao, int32_t nocc, const double *acc, const double *E, int nsums,
                     double *work, double *out, hipStream_t s)
{
    double *gram = work + gram_work_doubles(nocc);
    launch_gram_bound(C, nao, nocc, work, gram, s);
    hipLaunchKernelGGL(k_i8_bound, dim3(1), dim3(256), 0, s, acc, nao, gram, E, nsums, out);
}

}  // namespace dfjk
