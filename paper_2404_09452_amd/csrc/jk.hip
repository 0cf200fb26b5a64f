// One DF-J/K build on gfx950, from the resident whitened tensor B[f][P]
// (f = stored AO function pair of a significant shell pair, P = aux function,
// row length naux_pad):
//   1. D = 2 C C^T                           (C route only)
//   2. d_f = w_f D[mu_f][nu_f]               (w = 2 for a != b blocks, 1 for a == a)
//   3. c_P = sum_f d_f B[f][P]               split over f, fixed-order sum
//   4. J[mu_f][nu_f] = sum_P B[f][P] c_P     one wave per row f
//   5. X[mu][P][i] = sum_nu B[f(mu,nu)][P] C[nu][i]
//                                            gathered GEMM on FP64 MFMA, one
//                                            workgroup per (mu, 64 aux rows)
//   6. K = 2 X X^T (C route) or X B~^T (D route) on FP64 MFMA, lower tiles,
//      split-K into partial tiles summed in a fixed order
//   7. E_J = 1/2 sum_P c_P^2 (= 1/2 Tr DJ), E_K = -1/4 sum D K
// No floating-point atomics anywhere, so results are bitwise reproducible.
#include "dfjk_internal.h"
#include "gemm_f64.h"

namespace dfjk {

constexpr int kTileK = 128;      // syrk output tile
constexpr int kCSplitRows = 512; // f rows per partial of c

// ---------------------------------------------------------------------------
__global__ void k_fill(double *p, int64_t n, double v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
static void fill(double *p, int64_t n, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

// D = 2 C C^T, one thread per element of a 16x16 output block.
__global__ __launch_bounds__(256) void k_density(const double *__restrict__ C, int64_t nao, int32_t nocc,
                                                 double *__restrict__ D)
{
    __shared__ double Ca[16][65], Cb[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 16, n0 = (int64_t)blockIdx.x * 16;
    double s = 0.0;
    for (int i0 = 0; i0 < nocc; i0 += 64) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e / 64, c = e % 64;
            const bool ok = i0 + c < nocc;
            Ca[r][c] = (ok && m0 + r < nao) ? C[(m0 + r) * nocc + i0 + c] : 0.0;
            Cb[r][c] = (ok && n0 + r < nao) ? C[(n0 + r) * nocc + i0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 64; ++c) s += Ca[ty][c] * Cb[tx][c];
        __syncthreads();
    }
    if (m0 + ty < nao && n0 + tx < nao) D[(m0 + ty) * nao + n0 + tx] = 2.0 * s;
}

__global__ void k_gather_d(const double *__restrict__ D, int64_t nao, const int32_t *__restrict__ fmu,
                           const int32_t *__restrict__ fnu, const double *__restrict__ fw, int64_t nf,
                           int64_t nf_pad, double *__restrict__ d)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= nf_pad) return;
    d[f] = (f < nf) ? fw[f] * D[(int64_t)fmu[f] * nao + fnu[f]] : 0.0;
}

// cpart[s][P] = sum_{f in rows of split s} d_f B[f][P]
__global__ __launch_bounds__(256) void k_c_partial(const double *__restrict__ B, int64_t ld,
                                                   const double *__restrict__ d, int64_t nf_pad,
                                                   double *__restrict__ cpart)
{
    const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (P >= ld) return;
    const int64_t f0 = (int64_t)blockIdx.y * kCSplitRows;
    int64_t f1 = f0 + kCSplitRows;
    if (f1 > nf_pad) f1 = nf_pad;
    double s0 = 0.0, s1 = 0.0;
    int64_t f = f0;
    for (; f + 1 < f1; f += 2) {
        s0 += d[f] * B[f * ld + P];
        s1 += d[f + 1] * B[(f + 1) * ld + P];
    }
    if (f < f1) s0 += d[f] * B[f * ld + P];
    cpart[blockIdx.y * ld + P] = s0 + s1;
}

__global__ void k_c_reduce(const double *__restrict__ cpart, int nsplit, int64_t ld, double *__restrict__ c)
{
    const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (P >= ld) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += cpart[k * ld + P];
    c[P] = s;
}

// J_f = sum_P B[f][P] c_P; one wave per row.  Diagonal blocks hold both
// orientations as separate rows, so they write only their own element.
__global__ __launch_bounds__(256) void k_j_rows(const double *__restrict__ B, int64_t ld,
                                                const double *__restrict__ c, const int32_t *__restrict__ fmu,
                                                const int32_t *__restrict__ fnu, const double *__restrict__ fw,
                                                int64_t nf, int64_t nao, double *__restrict__ J)
{
    const int64_t f = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= nf) return;
    const double *row = B + f * ld;
    double s = 0.0;
    for (int64_t P = lane; P < ld; P += 64) s += row[P] * c[P];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const int64_t mu = fmu[f], nu = fnu[f];
        J[mu * nao + nu] = s;
        if (fw[f] > 1.5) J[nu * nao + mu] = s;
    }
}

// ---------------------------------------------------------------------------
// Half transform.  Workgroup (mu, 64-row P tile); wave w owns rows
// p0 + 16w .. +15 and every column block of 16 (up to 16 blocks per pass).
// The gathered coefficient rows C[nu_k][:] for 32 k at a time sit in LDS.
// MFMA: A = B[row_k][P] (lane: P = l%16, k = l/16), B = Cs[k][i]
// (lane: k = l/16, i = l%16); accumulator r holds row P = l/16 + 4r.

enum { OUT_F64 = 0, OUT_F32 = 1, OUT_BF16X2 = 2 };

struct HTArgs {
    const double *B;          // [f][ld]
    int64_t ld;               // naux_pad
    const double *C;          // [nao][ncol]
    int32_t ncol;
    const int32_t *hk_off, *hk_row, *hk_nu;
    void *X;                  // [nao][ld][ncol]
    void *Xlo;                // second plane for the BF16 split
};

constexpr int kHTK = 32;
constexpr int kHTCols = 256;

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x)
{
    unsigned int u = __float_as_uint(x);
    const unsigned int rounding = 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)((u + rounding) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

template <int OUT>
__global__ __launch_bounds__(256) void k_halftrans(HTArgs g)
{
    __shared__ double Cs[kHTK][kHTCols + 1];
    __shared__ int32_t rowS[kHTK];
    const int mu = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kb = g.hk_off[mu], ke = g.hk_off[mu + 1];
    const int64_t prow = p0 + 16 * wave + (lane & 15);

    for (int ic0 = 0; ic0 < g.ncol; ic0 += kHTCols) {
        const int width = min(kHTCols, g.ncol - ic0);
        const int nib = (width + 15) / 16;
        f64x4 acc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};
        for (int kc = kb; kc < ke; kc += kHTK) {
            for (int e = tid; e < kHTK * kHTCols; e += 256) {
                const int kk = e / kHTCols, i = e % kHTCols;
                double v = 0.0;
                if (kc + kk < ke && i < width) v = g.C[(int64_t)g.hk_nu[kc + kk] * g.ncol + ic0 + i];
                Cs[kk][i] = v;
            }
            if (tid < kHTK) rowS[tid] = (kc + tid < ke) ? g.hk_row[kc + tid] : -1;
            __syncthreads();
            double a[kHTK / 4];
#pragma unroll
            for (int ks = 0; ks < kHTK / 4; ++ks) {
                const int r = rowS[ks * 4 + (lane >> 4)];
                a[ks] = (r >= 0) ? g.B[(int64_t)r * g.ld + prow] : 0.0;
            }
#pragma unroll
            for (int ks = 0; ks < kHTK / 4; ++ks) {
                const double *cs = &Cs[ks * 4 + (lane >> 4)][lane & 15];
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < nib) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], cs[j * 16], acc[j], 0, 0, 0);
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j >= nib) break;
            const int col = ic0 + j * 16 + (lane & 15);
            if (col >= g.ncol) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t P = p0 + 16 * wave + (lane >> 4) + 4 * r;
                const int64_t o = ((int64_t)mu * g.ld + P) * g.ncol + col;
                if (OUT == OUT_F64) {
                    static_cast<double *>(g.X)[o] = acc[j][r];
                } else if (OUT == OUT_F32) {
                    static_cast<float *>(g.X)[o] = (float)acc[j][r];
                } else {
                    const float v = (float)acc[j][r];
                    const unsigned short hi = f32_to_bf16_rne(v);
                    const unsigned short lo = f32_to_bf16_rne(v - bf16_to_f32(hi));
                    static_cast<unsigned short *>(g.X)[o] = hi;
                    static_cast<unsigned short *>(g.Xlo)[o] = lo;
                }
            }
        }
    }
}

// Dense expansion for the D route: Bt[mu][P][nu] = B[f(mu,nu)][P] (0 elsewhere).
__global__ __launch_bounds__(256) void k_expand_B(const double *__restrict__ B, int64_t ld,
                                                  const int32_t *__restrict__ hk_off,
                                                  const int32_t *__restrict__ hk_row,
                                                  const int32_t *__restrict__ hk_nu, int64_t nao,
                                                  double *__restrict__ Bt)
{
    const int mu = blockIdx.y;
    const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (P >= ld) return;
    double *dst = Bt + ((int64_t)mu * ld + P) * nao;
    for (int64_t n = 0; n < nao; ++n) dst[n] = 0.0;
    for (int k = hk_off[mu]; k < hk_off[mu + 1]; ++k) dst[hk_nu[k]] = B[(int64_t)hk_row[k] * ld + P];
}

// ---------------------------------------------------------------------------
// Split-K reduction of the K tiles: K[m][n] = scale * sum_s partial[s][t][..]
// in a fixed order, mirrored for off-diagonal tiles, plus per-block partial
// sums of D[m][n] K[m][n] (weight 2 off the diagonal tiles) for E_K.
__global__ __launch_bounds__(256) void k_k_reduce(const double *__restrict__ part, int nsplit, int ntm,
                                                  int64_t nao, double scale, const double *__restrict__ D,
                                                  double *__restrict__ K, double *__restrict__ Epart)
{
    __shared__ double red[256];
    const int t = blockIdx.x;
    const int ntiles = ntm * (ntm + 1) / 2;
    int tm = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (tm * (tm + 1) / 2 > t) --tm;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int chunk = blockIdx.y;   // 16 rows of the tile per block
    double e = 0.0;
    for (int q = threadIdx.x; q < 16 * kTileK; q += 256) {
        const int row = chunk * 16 + q / kTileK, col = q % kTileK;
        const int64_t m = (int64_t)tm * kTileK + row, n = (int64_t)tn * kTileK + col;
        if (m >= nao || n >= nao) continue;
        const int64_t off = (int64_t)t * kTileK * kTileK + row * kTileK + col;
        double s = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t)sp * ntiles * kTileK * kTileK + off];
        s *= scale;
        K[m * nao + n] = s;
        double w = 1.0;
        if (tm != tn) {
            K[n * nao + m] = s;
            w = 2.0;
        }
        e += w * D[m * nao + n] * s;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) Epart[(int64_t)t * gridDim.y + chunk] = red[0];
}

__global__ __launch_bounds__(256) void k_energies(const double *__restrict__ c, int64_t naux,
                                                  const double *__restrict__ Epart, int64_t nEpart,
                                                  double *__restrict__ E)
{
    __shared__ double r1[256], r2[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < naux; i += 256) a += c[i] * c[i];
    for (int64_t i = threadIdx.x; i < nEpart; i += 256) b += Epart[i];
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r1[threadIdx.x] += r1[threadIdx.x + w];
            r2[threadIdx.x] += r2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        E[0] = 0.5 * r1[0];
        E[1] = -0.25 * r2[0];
    }
}

// ---------------------------------------------------------------------------

static int choose_ksplit(int ntiles, int64_t kdim)
{
    // aim for >= 1024 workgroups; every split a multiple of 16 in k
    int ns = (1024 + ntiles - 1) / ntiles;
    const int64_t maxs = kdim / 256;
    if (ns > maxs) ns = (int)(maxs > 0 ? maxs : 1);
    if (ns < 1) ns = 1;
    return ns;
}

BuildLayout build_layout(const Plan &p, int32_t nocc, int32_t precision, bool with_D)
{
    BuildLayout L{};
    L.nao = p.nao;
    L.naux_pad = p.naux_pad;
    L.nf = p.nf_pad;
    L.ncol = with_D ? p.nao : nocc;
    L.precision = precision;
    L.with_D = with_D;
    L.nsplit_c = (int)((p.nf_pad + kCSplitRows - 1) / kCSplitRows);
    L.ntile = (int)((p.nao + kTileK - 1) / kTileK);
    L.kdim = p.naux_pad * L.ncol;
    const int ntiles = L.ntile * (L.ntile + 1) / 2;
    L.nsplit_k = choose_ksplit(ntiles, L.kdim);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t o = off;
        off += bytes;
        return o;
    };
    L.o_D = take((size_t)p.nao * p.nao * 8);
    L.o_d = take((size_t)p.nf_pad * 8);
    L.o_cpart = take((size_t)L.nsplit_c * p.naux_pad * 8);
    L.o_c = take((size_t)p.naux_pad * 8);
    const size_t nx = (size_t)p.nao * L.kdim;
    const size_t esz = precision == DFJK_FP64 ? 8 : (precision == DFJK_MIXED_FP32 ? 4 : 2);
    L.o_X = take(nx * esz);
    L.o_Xlo = precision == DFJK_MIXED_BF16X3 ? take(nx * 2) : 0;
    L.o_Bfull = with_D ? take(nx * 8) : 0;
    L.o_Kpart = take((size_t)L.nsplit_k * ntiles * kTileK * kTileK * 8);
    L.o_Epart = take((size_t)ntiles * (kTileK / 16) * 8);
    L.bytes = align_up(off, 256);
    return L;
}

void launch_syrk_mixed(const BuildLayout &L, const void *X, const void *Xlo, double *part, hipStream_t s);

void launch_build(const Plan &p, const BuildLayout &L, const double *C, const double *Din, double *J,
                  double *K, double *E, char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    double *D = reinterpret_cast<double *>(scratch + L.o_D);
    double *dvec = reinterpret_cast<double *>(scratch + L.o_d);
    double *cpart = reinterpret_cast<double *>(scratch + L.o_cpart);
    double *cvec = reinterpret_cast<double *>(scratch + L.o_c);
    void *X = scratch + L.o_X;
    void *Xlo = L.o_Xlo ? scratch + L.o_Xlo : nullptr;
    double *Bt = L.o_Bfull ? reinterpret_cast<double *>(scratch + L.o_Bfull) : nullptr;
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    double *Epart = reinterpret_cast<double *>(scratch + L.o_Epart);

    // 1. density
    if (!L.with_D) {
        dim3 grid((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16));
        hipLaunchKernelGGL(k_density, grid, dim3(256), 0, s, C, nao, (int32_t)L.ncol, D);
    } else {
        (void)hipMemcpyAsync(D, Din, (size_t)nao * nao * 8, hipMemcpyDeviceToDevice, s);
    }
    // 2-4. J
    hipLaunchKernelGGL(k_gather_d, dim3((unsigned)((p.nf_pad + 255) / 256)), dim3(256), 0, s, D, nao, p.d.f_mu,
                       p.d.f_nu, p.d.f_w, p.nf, p.nf_pad, dvec);
    hipLaunchKernelGGL(k_c_partial, dim3((unsigned)((ld + 255) / 256), L.nsplit_c), dim3(256), 0, s, p.d.B, ld,
                       dvec, p.nf_pad, cpart);
    hipLaunchKernelGGL(k_c_reduce, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, s, cpart, L.nsplit_c, ld,
                       cvec);
    fill(J, nao * nao, 0.0, s);
    if (p.nf > 0)
        hipLaunchKernelGGL(k_j_rows, dim3((unsigned)((p.nf + 3) / 4)), dim3(256), 0, s, p.d.B, ld, cvec, p.d.f_mu,
                           p.d.f_nu, p.d.f_w, p.nf, nao, J);
    // 5. half transform
    HTArgs h{p.d.B, ld, L.with_D ? Din : C, (int32_t)L.ncol, p.d.hk_off, p.d.hk_row, p.d.hk_nu, X, Xlo};
    dim3 hgrid((unsigned)(ld / 64), (unsigned)nao);
    if (L.precision == DFJK_FP64) hipLaunchKernelGGL(k_halftrans<OUT_F64>, hgrid, dim3(256), 0, s, h);
    else if (L.precision == DFJK_MIXED_FP32) hipLaunchKernelGGL(k_halftrans<OUT_F32>, hgrid, dim3(256), 0, s, h);
    else hipLaunchKernelGGL(k_halftrans<OUT_BF16X2>, hgrid, dim3(256), 0, s, h);
    // 6. K
    const int ntiles = L.ntile * (L.ntile + 1) / 2;
    const int64_t ksplit = align_up((size_t)((L.kdim + L.nsplit_k - 1) / L.nsplit_k), 16);
    if (L.precision == DFJK_FP64) {
        GemmArgs g{};
        g.A = static_cast<const double *>(X); g.lda = L.kdim;
        if (L.with_D) {
            hipLaunchKernelGGL(k_expand_B, dim3((unsigned)((ld + 255) / 256), (unsigned)nao), dim3(256), 0, s,
                               p.d.B, ld, p.d.hk_off, p.d.hk_row, p.d.hk_nu, nao, Bt);
            g.B = Bt;
        } else {
            g.B = static_cast<const double *>(X);
        }
        g.ldb = L.kdim;
        g.M = g.N = nao;
        g.k_begin = 0; g.k_end = L.kdim; g.ksplit = ksplit;
        g.alpha = 1.0; g.lower = 1; g.partial = Kpart;
        gemm_f64<kTileK, false>(g, L.nsplit_k, s);
    } else {
        launch_syrk_mixed(L, X, Xlo, Kpart, s);
    }
    const double scale = L.with_D ? 1.0 : 2.0;
    hipLaunchKernelGGL(k_k_reduce, dim3(ntiles, kTileK / 16), dim3(256), 0, s, Kpart, L.nsplit_k, L.ntile, nao,
                       scale, D, K, Epart);
    // 7. energies
    hipLaunchKernelGGL(k_energies, dim3(1), dim3(256), 0, s, cvec, ld, Epart, (int64_t)ntiles * (kTileK / 16), E);
}

}  // namespace dfjk
