// One DF-J/K build on gfx950, from the resident whitened tensor B[f][P]
// (f = stored AO function pair of a significant shell pair, P = aux function,
// row length naux_pad):
//   1. D = 2 C C^T                           (C route only)
//   2. d_f = w_f D[mu_f][nu_f]               (w = 2 for a != b blocks, 1 for a == a)
//   3. c_P = sum_f d_f B[f][P]               split over f, fixed-order sum
//   4. J[mu_f][nu_f] = sum_P B[f][P] c_P     one wave per row f
//   5. X[mu][P][i] = sum_nu B[f(mu,nu)][P] C[nu][i]
//                                            gathered GEMM on FP64 MFMA, one
//                                            workgroup per (mu, 128 aux rows)
//   6. K = 2 X X^T (C route) or X B~^T (D route) on FP64 MFMA, lower tiles,
//      split-K into partial tiles summed in a fixed order
//   7. E_J = 1/2 sum_P c_P^2 (= 1/2 Tr DJ), E_K = -1/4 sum D K
// No floating-point atomics anywhere, so results are bitwise reproducible.
#include "dfjk_internal.h"
#include "gemm_f64.h"

namespace dfjk {


constexpr int kCSplitRows = 512; // f rows per partial of c
constexpr double kAutoSlabBytes = 48e9;  // automatic aux slab: slab-sized K buffers up to this

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

// D = scale C C^T, one thread per element of a 16x16 output block.
__global__ __launch_bounds__(256) void k_density(const double *__restrict__ C, int64_t nao, int32_t nocc,
                                                 double scale, double *__restrict__ D)
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
    if (m0 + ty < nao && n0 + tx < nao) D[(m0 + ty) * nao + n0 + tx] = scale * s;
}

void launch_density(const double *C, int64_t nao, int32_t nocc, double scale, double *D, hipStream_t s)
{
    hipLaunchKernelGGL(k_density, dim3((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16)), dim3(256), 0, s,
                       C, nao, nocc, scale, D);
}

__global__ void k_add(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
                      double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
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
#pragma unroll 4
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
#pragma unroll 8
    for (int k = 0; k < nsplit; ++k) s += cpart[k * ld + P];
    c[P] = s;
}

// J_f = sum_P B[f][P] c_P; one wave per row.  Diagonal blocks hold both
// orientations as separate rows, so they write only their own element.
__global__ __launch_bounds__(256) void k_j_rows(const double *__restrict__ B, int64_t ld,
                                                const double *__restrict__ c, const int32_t *__restrict__ fmu,
                                                const int32_t *__restrict__ fnu, const double *__restrict__ fw,
                                                int64_t nf, int64_t nao, int32_t accumulate, double *__restrict__ J)
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
        const double v = accumulate ? J[mu * nao + nu] + s : s;
        J[mu * nao + nu] = v;
        if (fw[f] > 1.5) J[nu * nao + mu] = v;
    }
}

// ---------------------------------------------------------------------------
// The same steps (density, zero-padded coefficients, J) for the molecules of a
// batch in shared launches, one per step: workgroup b of a step belongs to
// molecule m for blk_start[m] <= b < blk_start[m + 1] and runs what block
// b - blk_start[m] of that molecule's own launch runs, with the same
// arithmetic per element, so J and c are bitwise those of separate builds.
struct PreArgs {
    const double *C;          // nao x nocc orbitals
    double *D, *Cp, *J;       // density (2 C C^T), padded coefficients, J
    const int32_t *f_mu, *f_nu;
    const double *f_w, *B;
    double *dvec, *cpart, *cvec;
    int64_t nao, nf, nf_pad, ld;
    int32_t nocc, ldc, nsplit_c, pad_;
};
constexpr int kPreGroupMax = 16;
struct PreGroup {
    int32_t n;
    uint32_t blk_start[kPreGroupMax + 1];
    PreArgs a[kPreGroupMax];
};
static_assert(sizeof(PreGroup) <= 4096, "kernel arguments are limited to 4 KB");
enum { PRE_DENSITY, PRE_PAD, PRE_FILL_J, PRE_GATHER, PRE_CPART, PRE_CREDUCE, PRE_JROWS, PRE_STEPS };

__device__ __forceinline__ int pre_member(const PreGroup &g, unsigned &local)
{
    int m = 0;
    while (m + 1 < g.n && blockIdx.x >= g.blk_start[m + 1]) ++m;
    local = blockIdx.x - g.blk_start[m];
    return m;
}

// Workgroups of step `st` for one molecule (its own launch's grid, flattened
// x fastest).
static int64_t pre_blocks(int st, const PreArgs &a)
{
    switch (st) {
    case PRE_DENSITY: { const int64_t g = (a.nao + 15) / 16; return g * g; }
    case PRE_PAD: return ((a.nao + 1) * a.ldc + 255) / 256;
    case PRE_FILL_J: return (a.nao * a.nao + 255) / 256;
    case PRE_GATHER: return (a.nf_pad + 255) / 256;
    case PRE_CPART: return ((a.ld + 255) / 256) * a.nsplit_c;
    case PRE_CREDUCE: return (a.ld + 255) / 256;
    default: return (a.nf + 3) / 4;
    }
}

__global__ __launch_bounds__(256) void k_density_group(PreGroup g)
{
    unsigned local;
    const PreArgs &a = g.a[pre_member(g, local)];
    const unsigned gx = (unsigned)((a.nao + 15) / 16);
    __shared__ double Ca[16][65], Cb[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m0 = (int64_t)(local / gx) * 16, n0 = (int64_t)(local % gx) * 16;
    const int64_t nao = a.nao;
    const int nocc = a.nocc;
    double s = 0.0;
    for (int i0 = 0; i0 < nocc; i0 += 64) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int r = e / 64, c = e % 64;
            const bool ok = i0 + c < nocc;
            Ca[r][c] = (ok && m0 + r < nao) ? a.C[(m0 + r) * nocc + i0 + c] : 0.0;
            Cb[r][c] = (ok && n0 + r < nao) ? a.C[(n0 + r) * nocc + i0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int c = 0; c < 64; ++c) s += Ca[ty][c] * Cb[tx][c];
        __syncthreads();
    }
    if (m0 + ty < nao && n0 + tx < nao) a.D[(m0 + ty) * nao + n0 + tx] = 2.0 * s;
}

__global__ __launch_bounds__(256) void k_pad_fill_group(PreGroup g, int step)
{
    unsigned local;
    const PreArgs &a = g.a[pre_member(g, local)];
    const int64_t i = (int64_t)local * 256 + threadIdx.x;
    if (step == PRE_PAD) {
        if (i >= (a.nao + 1) * a.ldc) return;
        const int64_t r = i / a.ldc, c = i % a.ldc;
        a.Cp[i] = (r < a.nao && c < a.nocc) ? a.C[r * a.nocc + c] : 0.0;
    } else if (step == PRE_FILL_J) {
        if (i < a.nao * a.nao) a.J[i] = 0.0;
    } else {   // PRE_GATHER
        if (i >= a.nf_pad) return;
        a.dvec[i] = (i < a.nf) ? a.f_w[i] * a.D[(int64_t)a.f_mu[i] * a.nao + a.f_nu[i]] : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_c_partial_group(PreGroup g)
{
    unsigned local;
    const PreArgs &a = g.a[pre_member(g, local)];
    const unsigned gx = (unsigned)((a.ld + 255) / 256);
    const int64_t P = (int64_t)(local % gx) * 256 + threadIdx.x;
    const int64_t split = local / gx, ld = a.ld;
    if (P >= ld) return;
    const int64_t f0 = split * kCSplitRows;
    int64_t f1 = f0 + kCSplitRows;
    if (f1 > a.nf_pad) f1 = a.nf_pad;
    const double *__restrict__ d = a.dvec;
    const double *__restrict__ B = a.B;
    double s0 = 0.0, s1 = 0.0;
    int64_t f = f0;
#pragma unroll 4
    for (; f + 1 < f1; f += 2) {
        s0 += d[f] * B[f * ld + P];
        s1 += d[f + 1] * B[(f + 1) * ld + P];
    }
    if (f < f1) s0 += d[f] * B[f * ld + P];
    a.cpart[split * ld + P] = s0 + s1;
}

__global__ __launch_bounds__(256) void k_c_reduce_group(PreGroup g)
{
    unsigned local;
    const PreArgs &a = g.a[pre_member(g, local)];
    const int64_t P = (int64_t)local * 256 + threadIdx.x;
    if (P >= a.ld) return;
    double s = 0.0;
#pragma unroll 8
    for (int k = 0; k < a.nsplit_c; ++k) s += a.cpart[k * a.ld + P];
    a.cvec[P] = s;
}

__global__ __launch_bounds__(256) void k_j_rows_group(PreGroup g)
{
    unsigned local;
    const PreArgs &a = g.a[pre_member(g, local)];
    const int64_t f = (int64_t)local * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (f >= a.nf) return;
    const double *row = a.B + f * a.ld;
    double s = 0.0;
    for (int64_t P = lane; P < a.ld; P += 64) s += row[P] * a.cvec[P];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        const int64_t mu = a.f_mu[f], nu = a.f_nu[f];
        a.J[mu * a.nao + nu] = s;
        if (a.f_w[f] > 1.5) a.J[nu * a.nao + mu] = s;
    }
}

// The steps in order, each as shared launches of up to kPreGroupMax molecules.
static void launch_pre_groups(const std::vector<PreArgs> &as, hipStream_t s)
{
    for (int st = 0; st < PRE_STEPS; ++st) {
        for (size_t first = 0; first < as.size(); first += kPreGroupMax) {
            PreGroup g{};
            int64_t total = 0;
            for (size_t i = first; i < as.size() && g.n < kPreGroupMax; ++i) {
                g.blk_start[g.n] = (uint32_t)total;
                g.a[g.n++] = as[i];
                total += pre_blocks(st, as[i]);
            }
            g.blk_start[g.n] = (uint32_t)total;
            if (total <= 0) continue;
            const dim3 grid((unsigned)total), block(256);
            switch (st) {
            case PRE_DENSITY: hipLaunchKernelGGL(k_density_group, grid, block, 0, s, g); break;
            case PRE_PAD:
            case PRE_FILL_J:
            case PRE_GATHER: hipLaunchKernelGGL(k_pad_fill_group, grid, block, 0, s, g, st); break;
            case PRE_CPART: hipLaunchKernelGGL(k_c_partial_group, grid, block, 0, s, g); break;
            case PRE_CREDUCE: hipLaunchKernelGGL(k_c_reduce_group, grid, block, 0, s, g); break;
            default: hipLaunchKernelGGL(k_j_rows_group, grid, block, 0, s, g); break;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Half transform.  MFMA operands: A = B[row_k][P] (lane: P = l%16,
// k = l/16), B = Cs[k][i] (lane: k = l/16, i = l%16); accumulator r holds
// row P = l/16 + 4r.

enum { OUT_F64 = 0, OUT_F32 = 1, OUT_BF16X2 = 2, OUT_I8 = 3 };
typedef double f64x2 __attribute__((ext_vector_type(2)));

struct HTArgs {
    const double *B;          // [f][ld]
    int64_t ld;               // naux_pad
    const double *C;          // [nao + 1][ldc]: coefficients zero-padded to ldc columns, row nao zero
    int32_t ncol;             // columns of the coefficients
    int32_t ldc;
    const int32_t *hk_off, *hk_row, *hk_nu;   // partner lists, each padded to a multiple of kHtChunk
    void *X;                  // [nao][plen][ncol]: aux rows p_begin .. p_begin + plen - 1
                              // (int8 slices: [nao][kdim/64][5][64], see kI8Slices)
    void *Xlo;                // second plane for the BF16 split; block scales for int8
    int64_t p_begin, plen;    // aux slab (multiples of 128)
    const int32_t *order;     // blockIdx.y -> AO function (longest list first)
    int32_t nslice;           // int8 slices written (the rest of each chunk is left as it was)
};


__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x)
{
    unsigned int u = __float_as_uint(x);
    const unsigned int rounding = 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)((u + rounding) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// LDS of one k chunk of the half transform: kHtChunk rows of the 128-wide B
// tile (the MFMA A operand, LDA apart), then kHtChunk rows of the pass's NCOL
// coefficient columns (LDC apart).  The row pitches put the four k rows that
// one fragment read touches on alternating halves of the banks.
template <int NCOL> struct HtLds {
    static constexpr int PAD = (16 - NCOL % 32 + 32) % 32;
    static constexpr int LDC = NCOL + PAD;
    static constexpr int LDA = 128 + 16;
    static constexpr int DOUBLES = kHtChunk * (LDA + LDC);
};

// Int8 output of one half-transform workgroup (mu, 128 aux rows p0.., the
// column pass ic0.. of width w = min(NCOL, ncol - ic0), stored w_e = w
// rounded up to even wide).  Contraction index inside the slab:
//   k = plen * ic0 + (P - p_begin) * w_e + (col - ic0),
// so the workgroup owns 128 w_e / 256 whole scale blocks and one contiguous
// byte range of the row (chunks of 64 k, five slices each).  Per block: the
// largest |x| (LDS atomics on the bit pattern, which orders like the value
// for non-negative doubles), e = the least exponent with 2^e > |x|max
// 128/127, the scale 2^e to g.Xlo; then x 2^-e = sum_s a_s 2^{-7(s+1)} by
// repeated rounding, every step exact in FP64 (a_0 = rint(128 x 2^-e) in
// [-127, 127], later a_s in [-64, 64]); slices 0 .. nslice - 1 are stored
// (four for int8_fast, whose K never reads a_4).  The pad column stores zeros.
// Slicing runs from LDS, 32 aux rows at a time: the two waves that hold them
// write their FP64 values to the first operand buffer in k order, then every
// thread slices four consecutive k and stores one 4-byte word per slice, so
// the registers of the accumulators are the only large live state.  The
// block maxima and exponents sit at the end of the second buffer.
template <int NIB>
__device__ __forceinline__ void store_i8(const HTArgs &g, const f64x4 (&acc)[NIB], double *st,
                                         unsigned char *tab, int mu, int64_t p0, int ic0, int tid, int lane,
                                         int wave, int kl)
{
    constexpr int NCOL = NIB * 16;
    static_assert(32 * NCOL * 8 <= HtLds<NCOL>::DOUBLES * 8, "32 rows of FP64 must fit a buffer");
    static_assert(128 * 12 <= HtLds<NCOL>::DOUBLES * 8, "block tables must fit a buffer");
    unsigned long long *bmax = reinterpret_cast<unsigned long long *>(tab);
    int *bexp = reinterpret_cast<int *>(tab + 128 * 8);
    const int w = min(NCOL, g.ncol - ic0), we = w + (w & 1);
    const int64_t kbase = g.plen * ic0 + (p0 - g.p_begin) * we;     // a multiple of kI8Block
    const int64_t kdim = g.plen * (int64_t)(g.ncol + (g.ncol & 1));
    const int64_t nblk = kdim / kI8Block;
    __syncthreads();   // the k loop's LDS reads are done
    if (tid < 128) bmax[tid] = 0ull;
    __syncthreads();
    // Block maxima.  A lane's values of one r lie in one aux row, whose we <=
    // 160 k span at most two blocks (lo, hi); the 16 lanes of that row (one
    // DPP row, lane & 15) reduce both by butterfly, then one lane of each row
    // updates the two blocks' maxima in LDS.
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row0 = (16 * wave + kl + 4 * r) * we;
        const int blo = row0 / kI8Block;
        double mlo = 0.0, mhi = 0.0;
#pragma unroll
        for (int j = 0; j < NIB; ++j) {
            const int c = j * 16 + (lane & 15);
            const double v = c < w ? fabs(acc[j][r]) : 0.0;
            if ((row0 + c) / kI8Block == blo) mlo = fmax(mlo, v);
            else mhi = fmax(mhi, v);
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            mlo = fmax(mlo, __shfl_xor(mlo, o, 16));
            mhi = fmax(mhi, __shfl_xor(mhi, o, 16));
        }
        if ((lane & 15) == 0) {
            atomicMax(&bmax[blo], (unsigned long long)__double_as_longlong(mlo));
            if ((row0 + we - 1) / kI8Block != blo)
                atomicMax(&bmax[blo + 1], (unsigned long long)__double_as_longlong(mhi));
        }
    }
    __syncthreads();
    const int nb = 128 * we / kI8Block;
    if (tid < nb) {
        const double m = __longlong_as_double((long long)bmax[tid]);
        const int e = m > 0.0 ? ilogb(m * (128.0 / 127.0)) + 1 : 0;
        bexp[tid] = e;
        static_cast<double *>(g.Xlo)[(int64_t)mu * nblk + kbase / kI8Block + tid] = ldexp(1.0, e);
    }
    unsigned char *dst = static_cast<unsigned char *>(g.X) + (int64_t)mu * kdim * kI8Slices +
                         (kbase / kI8Chunk) * (kI8Chunk * kI8Slices);
    const int qk = 32 * we;                                            // k of 32 aux rows
    for (int q = 0; q < 4; ++q) {
        __syncthreads();   // exponents written; the previous quarter's values read
        if ((wave >> 1) == q) {
#pragma unroll
            for (int j = 0; j < NIB; ++j) {
                const int c = j * 16 + (lane & 15);
                if (c >= we) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    st[(16 * (wave & 1) + kl + 4 * r) * we + c] = c < w ? acc[j][r] : 0.0;
            }
        }
        __syncthreads();
        for (int it = tid; it < qk / 4; it += 512) {
            const int kq = 4 * it, k = q * qk + kq;                  // k within the workgroup's range
            const int e = bexp[k / kI8Block];                        // four k share a block
            double t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] = ldexp(st[kq + u], -e);
            unsigned char *d = dst + (k / kI8Chunk) * (kI8Chunk * kI8Slices) + (k % kI8Chunk);
#pragma unroll
            for (int sl = 0; sl < kI8Slices; ++sl) {
                if (sl >= g.nslice) break;
                unsigned int word = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    t[u] *= 128.0;
                    const double a = rint(t[u]);
                    t[u] -= a;
                    word |= (unsigned int)(unsigned char)(signed char)(int)a << (8 * u);
                }
                *reinterpret_cast<unsigned int *>(d + sl * kI8Chunk) = word;
            }
        }
    }
}

// s_waitcnt immediate for vmcnt(0) (gfx9 encoding; expcnt and lgkmcnt at
// their maxima do not wait), issued through the builtin so the compiler's own
// wait insertion knows the loads have retired.
constexpr int kHtWaitVm0 = 0 | (7 << 4) | (15 << 8);

// Workgroup (mu, 128-row P tile, column pass of NIB*16 columns) of eight
// waves, each 16 aux rows x NIB fragments: X[mu][P][i] = sum over mu's
// partners k of B[row_k][P] C[nu_k][i].  The partners run in chunks of
// kHtChunk; each chunk's B rows (1 KB each) and coefficient rows move from
// global memory straight into one of two LDS buffers (global_load_lds, 16
// bytes a lane, no registers), the next chunk in flight while the MFMAs use
// the current one, one barrier per chunk.  Wave w brings rows 2w and 2w+1 of
// both operands; the partner indices of the chunk after next are loaded
// into a register (lane l: entry l of the chunk) with the DMA, so issuing a
// chunk never waits on an index load.  The padded partner lists make every
// chunk whole; the padded coefficients keep every 16-byte piece in bounds.
template <int OUT, int NIB>
__device__ __forceinline__ void halftrans_tile(HTArgs g, unsigned bx, unsigned by, unsigned bz)
{
    constexpr int KC = kHtChunk, NCOL = NIB * 16;
    constexpr int LDA = HtLds<NCOL>::LDA, LDC = HtLds<NCOL>::LDC;
    constexpr int NPR = (NCOL + 127) / 128;             // DMA instructions per coefficient row
    // two chunk buffers as separate arrays: the compiler then tells a read of
    // one from a DMA into the other and does not wait for unrelated loads
    __shared__ __attribute__((aligned(1024))) double sb0[HtLds<NCOL>::DOUBLES];
    __shared__ __attribute__((aligned(1024))) double sb1[HtLds<NCOL>::DOUBLES];
    const int mu = g.order[by];
    const int64_t p0 = g.p_begin + (int64_t)bx * 128;
    const int ic0 = bz * NCOL;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kb = g.hk_off[mu], ke = g.hk_off[mu + 1];
    const int nch = (ke - kb) / KC;
    const int kl = lane >> 4;   // k within an MFMA step

    f64x4 acc[NIB];
#pragma unroll
    for (int j = 0; j < NIB; ++j) acc[j] = f64x4{0.0, 0.0, 0.0, 0.0};

    // partner indices of chunk ci (lane l: entry l % 16; past the list: its last entry)
    int rowv = 0, nuv = 0;
    auto load_idx = [&](int ci) {
        const int k = min(kb + ci * KC + (lane & 15), ke - 1);
        rowv = g.hk_row[k];
        nuv = g.hk_nu[k];
    };
    auto dma = [&](double *buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = 2 * wave + i;
            const int row = __builtin_amdgcn_readlane(rowv, r);
            const int nu = __builtin_amdgcn_readlane(nuv, r);
            __builtin_amdgcn_global_load_lds(
                (const void *)(g.B + (int64_t)row * g.ld + p0 + 2 * lane),
                (__attribute__((address_space(3))) void *)(buf + r * LDA), 16, 0, 0);
#pragma unroll
            for (int q = 0; q < NPR; ++q)
                if (q * 128 + 2 * lane < NCOL)
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(g.C + (int64_t)nu * g.ldc + ic0 + q * 128 + 2 * lane),
                        (__attribute__((address_space(3))) void *)(buf + KC * LDA + r * LDC + q * 128), 16, 0, 0);
        }
    };
    // one chunk: wait for its DMA (every wave's, through the barrier, which
    // also tells that every wave has finished reading `nxt`), start the next
    // chunk's DMA into `nxt`, then the MFMAs on `cur`
    auto step = [&](const double *cur, double *nxt, int c) {
        __builtin_amdgcn_s_waitcnt(kHtWaitVm0);
        __syncthreads();
        if (c + 1 < nch) {
            dma(nxt);
            load_idx(c + 2);
        }
        __builtin_amdgcn_sched_barrier(0);
        const double *as = cur + kl * LDA + 16 * wave + (lane & 15);
        const double *cs = cur + KC * LDA + kl * LDC + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            const double a = as[ks * 4 * LDA];
#pragma unroll
            for (int j = 0; j < NIB; ++j)
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cs[ks * 4 * LDC + j * 16], acc[j], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    if (nch > 0) {
        load_idx(0);
        dma(sb0);
        load_idx(1);
        for (int c = 0; c < nch; c += 2) {
            step(sb0, sb1, c);
            if (c + 1 < nch) step(sb1, sb0, c + 1);
        }
    }

    if constexpr (OUT == OUT_I8) {
        store_i8(g, acc, sb0, reinterpret_cast<unsigned char *>(sb1), mu, p0, ic0, tid, lane, wave, kl);
        return;
    }
#pragma unroll
    for (int j = 0; j < NIB; ++j) {
        const int col = ic0 + j * 16 + (lane & 15);
        if (col >= g.ncol) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t P = p0 + 16 * wave + kl + 4 * r;
            const int64_t o = ((int64_t)mu * g.plen + (P - g.p_begin)) * g.ncol + col;
            const double v64 = acc[j][r];
            if (OUT == OUT_F64) {
                __builtin_nontemporal_store(v64, static_cast<double *>(g.X) + o);
            } else if (OUT == OUT_F32) {
                __builtin_nontemporal_store((float)v64, static_cast<float *>(g.X) + o);
            } else {
                const float v = (float)v64;
                const unsigned short hi = f32_to_bf16_rne(v);
                const unsigned short lo = f32_to_bf16_rne(v - bf16_to_f32(hi));
                static_cast<unsigned short *>(g.X)[o] = hi;
                static_cast<unsigned short *>(g.Xlo)[o] = lo;
            }
        }
    }
}

template <int OUT, int NIB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_halftrans(HTArgs g)
{
    halftrans_tile<OUT, NIB>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Half transforms of several molecules (the same output and fragment count)
// in one launch: workgroup b runs workgroup b - blk_start[m] of molecule m's own
// grid (gx P tiles fastest, then gy AO functions, then column passes), with
// its arguments passed by value, so small molecules share the chip.
constexpr int kHtGroupMax = 16;
struct HtGroup {
    int32_t n;
    uint32_t blk_start[kHtGroupMax + 1];
    uint32_t gx[kHtGroupMax], gy[kHtGroupMax];
    HTArgs g[kHtGroupMax];
};
static_assert(sizeof(HtGroup) <= 4096, "kernel arguments are limited to 4 KB");

template <int OUT, int NIB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_halftrans_group(HtGroup grp)
{
    int m = 0;
    while (m + 1 < grp.n && blockIdx.x >= grp.blk_start[m + 1]) ++m;
    const unsigned local = blockIdx.x - grp.blk_start[m];
    const unsigned bx = local % grp.gx[m], rest = local / grp.gx[m];
    halftrans_tile<OUT, NIB>(grp.g[m], bx, rest % grp.gy[m], rest / grp.gy[m]);
}

// Coefficients for the half transform: Cp[nao + 1][ldc] with C in the first
// ncol columns of the first nao rows and zeros elsewhere.
__global__ __launch_bounds__(256) void k_pad_coef(const double *__restrict__ C, int64_t nao, int32_t ncol,
                                                  int32_t ldc, double *__restrict__ Cp)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (nao + 1) * ldc) return;
    const int64_t r = i / ldc, c = i % ldc;
    Cp[i] = (r < nao && c < ncol) ? C[r * ncol + c] : 0.0;
}

template <int OUT>
static void launch_halftrans(const HTArgs &h, int64_t nao, hipStream_t s)
{
    const int nib = ht_pass_frags(h.ncol);
    dim3 grid((unsigned)(h.plen / 128), (unsigned)nao, (unsigned)ht_passes(h.ncol));
#define HT_CASE(N) \
    case N: hipLaunchKernelGGL((k_halftrans<OUT, N>), grid, dim3(512), 0, s, h); break;
    switch (nib) {
        HT_CASE(1) HT_CASE(2) HT_CASE(3) HT_CASE(4) HT_CASE(5) HT_CASE(6) HT_CASE(7) HT_CASE(8)
        HT_CASE(9) HT_CASE(10)
    }
#undef HT_CASE
}
static_assert(kHtMaxFrag == 10, "launch_halftrans instantiates 1..kHtMaxFrag fragments");

// Half transforms of several molecules with output OUT (FP64 or int8
// slices): those with the same fragment count share launches of
// k_halftrans_group (up to kHtGroupMax each).
template <int OUT>
static void launch_halftrans_groups(const std::vector<std::pair<HTArgs, int64_t>> &hs, hipStream_t s)
{
    for (int nib = 1; nib <= kHtMaxFrag; ++nib) {
        HtGroup grp{};
        int64_t total = 0;
        auto flush = [&]() {
            if (grp.n == 0) return;
            grp.blk_start[grp.n] = (uint32_t)total;
#define HT_CASE(N) \
    case N: hipLaunchKernelGGL((k_halftrans_group<OUT, N>), dim3((unsigned)total), dim3(512), 0, s, grp); break;
            switch (nib) {
                HT_CASE(1) HT_CASE(2) HT_CASE(3) HT_CASE(4) HT_CASE(5) HT_CASE(6) HT_CASE(7) HT_CASE(8)
                HT_CASE(9) HT_CASE(10)
            }
#undef HT_CASE
            grp = HtGroup{};
            total = 0;
        };
        for (const auto &e : hs) {
            const HTArgs &h = e.first;
            if (ht_pass_frags(h.ncol) != nib) continue;
            const int64_t gx = h.plen / 128, gy = e.second, gz = ht_passes(h.ncol);
            const int64_t nb = gx * gy * gz;
            if (nb <= 0) continue;
            if (grp.n == kHtGroupMax || total + nb > (int64_t)UINT32_MAX / 2) flush();
            grp.blk_start[grp.n] = (uint32_t)total;
            grp.gx[grp.n] = (uint32_t)gx;
            grp.gy[grp.n] = (uint32_t)gy;
            grp.g[grp.n++] = h;
            total += nb;
        }
        flush();
    }
}

static void dispatch_halftrans(int precision, const HTArgs &h, int64_t nao, hipStream_t s)
{
    switch (precision) {
    case DFJK_FP64: launch_halftrans<OUT_F64>(h, nao, s); break;
    case DFJK_MIXED_FP32: launch_halftrans<OUT_F32>(h, nao, s); break;
    case DFJK_MIXED_BF16X3: launch_halftrans<OUT_BF16X2>(h, nao, s); break;
    default: launch_halftrans<OUT_I8>(h, nao, s); break;
    }
}

// Dense expansion for the D route: Bt[mu][P][nu] = B[f(mu,nu)][P] (0 elsewhere).
__global__ __launch_bounds__(256) void k_expand_B(const double *__restrict__ B, int64_t ld,
                                                  const int32_t *__restrict__ hk_off,
                                                  const int32_t *__restrict__ hk_row,
                                                  const int32_t *__restrict__ hk_nu, int64_t nao,
                                                  int64_t p_begin, int64_t plen, double *__restrict__ Bt)
{
    const int mu = blockIdx.y;
    const int64_t pl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pl >= plen) return;
    const int64_t P = p_begin + pl;
    double *dst = Bt + ((int64_t)mu * plen + pl) * nao;
    for (int64_t n = 0; n < nao; ++n) dst[n] = 0.0;
    for (int k = hk_off[mu]; k < hk_off[mu + 1]; ++k)
        if (hk_nu[k] < nao) dst[hk_nu[k]] = B[(int64_t)hk_row[k] * ld + P];   // padding entries name row nao
}

// [U | W] = [C + C0 | C - C0] (nao x 2 nocc): 2(C C^T - C0 C0^T) = U W^T + W U^T.
__global__ void k_uw(const double *__restrict__ C, const double *__restrict__ C0, int64_t nao, int32_t nocc,
                     double *__restrict__ U, double *__restrict__ W)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nao * nocc) return;
    const double c = C[e], c0 = C0[e];
    U[e] = c + c0;
    W[e] = c - c0;
}

// Incremental K: K = K0 + G + G^T with G = X_U X_W^T held as split-K partial
// tiles over every 128x128 tile (rectangular order t = tm + tn * ntm).  One
// block per lower tile and 16-row chunk sums both G[m][n] and G[n][m] in a
// fixed order, writes K symmetric, and sums D o K for E_K.
__global__ __launch_bounds__(256) void k_k_reduce_delta(const double *__restrict__ part, int nsplit, int ntm,
                                                        int64_t nao, const double *__restrict__ K0,
                                                        const double *__restrict__ D, double *__restrict__ K,
                                                        double *__restrict__ Epart)
{
    __shared__ double red[256];
    const int t = blockIdx.x;
    int tm = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (tm * (tm + 1) / 2 > t) --tm;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    const int64_t tile_mn = tm + (int64_t)tn * ntm, tile_nm = tn + (int64_t)tm * ntm;
    const int64_t nt = (int64_t)ntm * ntm, TT = (int64_t)kTileK * kTileK;
    const int chunk = blockIdx.y;
    double e = 0.0;
    for (int q = threadIdx.x; q < 16 * kTileK; q += 256) {
        const int row = chunk * 16 + q / kTileK, col = q % kTileK;
        const int64_t m = (int64_t)tm * kTileK + row, n = (int64_t)tn * kTileK + col;
        if (m >= nao || n >= nao || n > m) continue;
        double g1 = 0.0, g2 = 0.0;
#pragma unroll 8
        for (int sp = 0; sp < nsplit; ++sp) {
            g1 += part[(sp * nt + tile_mn) * TT + row * kTileK + col];
            g2 += part[(sp * nt + tile_nm) * TT + col * kTileK + row];
        }
        const double v = K0[m * nao + n] + (g1 + g2);
        K[m * nao + n] = v;
        double w = 1.0;
        if (m != n) {
            K[n * nao + m] = v;
            w = 2.0;
        }
        e += w * D[m * nao + n] * v;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) Epart[(int64_t)t * gridDim.y + chunk] = red[0];
}

// ---------------------------------------------------------------------------
// Split-K reduction of the K tiles: K[m][n] = scale * sum_s partial[s][t][..]
// in a fixed order, mirrored for off-diagonal tiles, plus per-block partial
// sums of D[m][n] K[m][n] (weight 2 off the diagonal tiles) for E_K.
// Rows of a tile per reduction workgroup: small enough that the grid has
// many workgroups (each lane sums its splits in turn, so the loads of many
// lanes in flight hide their latency).
constexpr int kReduceRows = 4;
constexpr int reduce_chunks(int T) { return T / kReduceRows; }

__device__ __forceinline__ void reduce_tile(const double *__restrict__ part, int nsplit, int ntm, int T, int64_t nao,
                                            double scale, const double *__restrict__ D, double *__restrict__ K,
                                            double *__restrict__ Epart, const int t, const int chunk)
{
    __shared__ double red[256];
    const int ntiles = ntm * (ntm + 1) / 2;
    int tm = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (tm * (tm + 1) / 2 > t) --tm;
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    const int tn = t - tm * (tm + 1) / 2;
    double e = 0.0;
    for (int q = threadIdx.x; q < kReduceRows * T; q += 256) {
        const int row = chunk * kReduceRows + q / T, col = q % T;
        const int64_t m = (int64_t)tm * T + row, n = (int64_t)tn * T + col;
        // the upper half of a diagonal tile is mirrored from its lower half
        if (m >= nao || n >= nao || n > m) continue;
        const int64_t off = (int64_t)t * T * T + row * T + col;
        double s = 0.0;
#pragma unroll 8
        for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t)sp * ntiles * T * T + off];
        s *= scale;
        K[m * nao + n] = s;
        double w = 1.0;
        if (m != n) {
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
    if (threadIdx.x == 0) Epart[(int64_t)t * reduce_chunks(T) + chunk] = red[0];
}

// block (t, chunk): lower tile t (T wide), rows kReduceRows chunk onwards
__global__ __launch_bounds__(256) void k_k_reduce(const double *__restrict__ part, int nsplit, int ntm, int T,
                                                  int64_t nao, double scale, const double *__restrict__ D,
                                                  double *__restrict__ K, double *__restrict__ Epart)
{
    reduce_tile(part, nsplit, ntm, T, nao, scale, D, K, Epart, blockIdx.x, blockIdx.y);
}

// Grouped reduction for a batch: blocks blk_start[p] .. blk_start[p+1]-1 reduce
// molecule p, whose tiles are T[p] wide; the grid has reduce_chunks(kTileK)
// chunks in y (the most any width needs) and molecule p uses the first
// reduce_chunks(T[p]).  Descriptors by value.
constexpr int kReduceGroupMax = 16;
struct ReduceGroup {
    int32_t n;
    int32_t blk_start[kReduceGroupMax + 1];
    int32_t nsplit[kReduceGroupMax], ntm[kReduceGroupMax], T[kReduceGroupMax];
    int64_t nao[kReduceGroupMax];
    const double *part[kReduceGroupMax], *D[kReduceGroupMax];
    double *K[kReduceGroupMax], *Epart[kReduceGroupMax];
};

__global__ __launch_bounds__(256) void k_k_reduce_grouped(ReduceGroup grp, double scale)
{
    const int b = blockIdx.x;
    int p = 0;
    while (p + 1 < grp.n && b >= grp.blk_start[p + 1]) ++p;
    if ((int)blockIdx.y >= reduce_chunks(grp.T[p])) return;   // past this molecule's rows
    reduce_tile(grp.part[p], grp.nsplit[p], grp.ntm[p], grp.T[p], grp.nao[p], scale, grp.D[p], grp.K[p],
                grp.Epart[p], b - grp.blk_start[p], blockIdx.y);
}

__device__ __forceinline__ void energies_body(const double *__restrict__ c, int64_t naux,
                                              const double *__restrict__ Epart, int64_t nEpart, double fk,
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
        E[1] = fk * r2[0];
    }
}

__global__ __launch_bounds__(256) void k_energies(const double *__restrict__ c, int64_t naux,
                                                  const double *__restrict__ Epart, int64_t nEpart, double fk,
                                                  double *__restrict__ E)
{
    energies_body(c, naux, Epart, nEpart, fk, E);
}

// one block per molecule of a batch
constexpr int kEnergyGroupMax = 64;
struct EnergyGroup {
    const double *c[kEnergyGroupMax], *Epart[kEnergyGroupMax];
    int64_t naux[kEnergyGroupMax], nEpart[kEnergyGroupMax];
    double *E[kEnergyGroupMax];
};

__global__ __launch_bounds__(256) void k_energies_grouped(EnergyGroup grp, double fk)
{
    const int p = blockIdx.x;
    energies_body(grp.c[p], grp.naux[p], grp.Epart[p], grp.nEpart[p], fk, grp.E[p]);
}

// ---------------------------------------------------------------------------

// Split-K count for the K contraction: the largest count whose workgroups
// (two per CU for these kernels) fit in one round, so no nearly empty last
// round idles the chip; at least 256 k values per split.
int mixed_nsplit(int64_t nao, int64_t kdim, bool lower, int num_cus);
int i8_nsplit(int64_t nao, int64_t kdim, bool lower, int num_cus);
void launch_gemm_i8(bool lower, const void *A, const double *sA, const void *B, const double *sB, int64_t nao,
                    int64_t kdim, int nsplit, bool fast, double *part, hipStream_t s);
void launch_gemm_i8_group(bool fast, int n, const void *const *X, const double *const *sX, const int64_t *nao,
                          const int64_t *kdim, const int *nsplit, double *const *part, hipStream_t s);

static int choose_ksplit(int ntiles, int64_t kdim, int num_cus, int per_cu = 2)
{
    const int slots = per_cu * (num_cus > 0 ? num_cus : 256);
    int ns = ntiles >= slots ? 1 : slots / ntiles;
    const int64_t maxs = kdim / 256;
    if (ns > maxs) ns = (int)(maxs > 0 ? maxs : 1);
    if (ns < 1) ns = 1;
    return ns;
}

static int xcd_round(int ns) { return ns >= kXcds ? ns / kXcds * kXcds : ns; }

BuildLayout build_layout(const Plan &p, int32_t nocc, int32_t precision, bool with_D, bool delta, int nsplit,
                         bool allow_overlap, int64_t force_slab, int ktile)
{
    BuildLayout L{};
    L.nao = p.nao;
    L.naux_pad = p.naux_pad;
    L.nf = p.nf_pad;
    L.ncol = with_D ? p.nao : nocc;
    L.precision = precision;
    L.with_D = with_D;
    L.nsplit_c = (int)((p.nf_pad + kCSplitRows - 1) / kCSplitRows);
    // The FP64 syrk (C and density routes) may run on 64-wide tiles, whose
    // partials and reduction then use that width: less of its work above the
    // diagonal or past nao.  The autotuner's choice for the shape, or the
    // caller's, wins; otherwise 64 when the 128-wide tiles would execute over
    // 14% more products (the 64-wide kernel sustains about 70% of the FP64
    // MFMA peak, the 128-wide one 80%).  Mixed precision, the increment and
    // batches keep 128.
    L.ktile = kTileK;
    if (precision == DFJK_FP64 && !delta) {
        int kt = ktile != 0 ? ktile : p.k_tile;
        if (kt == 0 && nsplit == 0 && !with_D) {
            const auto it = p.tuned_ktile.find((int64_t)nocc * 4 + precision);
            if (it != p.tuned_ktile.end()) kt = it->second;
        }
        if (kt == 0) {
            auto executed = [&](int64_t t) { const int64_t n = (p.nao + t - 1) / t; return n * (n + 1) / 2 * t * t; };
            if ((double)executed(kTileK) > 1.14 * (double)executed(64)) kt = 64;
        }
        if (kt == 64 || kt == 96) L.ktile = kt;
    }
    L.ntile = (int)((p.nao + L.ktile - 1) / L.ktile);
    L.delta = delta;
    // aux slab of the K build: X = nao x slab x ncol elements per operand
    // bytes of X per element (both BF16 planes; int8 slices plus block scales)
    const double esz = precision == DFJK_FP64 ? 8.0
                     : precision == DFJK_MIXED_FP32 ? 4.0
                     : precision == DFJK_MIXED_BF16X3 ? 4.0 : kI8Slices + 8.0 / kI8Block;
    // automatic: the largest multiple of 128 whose slab-sized buffers (X, its low part,
    // the expanded B of the density route, the second operand of the increment) stay
    // within kAutoSlabBytes
    // Overlapped slabs (C route): when the K build needs several aux slabs, the
    // half transform of slab s + 1 runs on a second stream while the K GEMM of
    // slab s runs, into the other of two X buffers (the automatic slab is
    // sized for both).  A molecule that fits one slab is not cut in two: at
    // 2,816 aux that saved 1.5% of an FP64 build, lost 3% in FP32, and the
    // GEMM shares the chip with the half transform while they overlap.  The
    // int8 GEMM, bound by operand traffic through L2, runs slabs in turn:
    // beside the half transform the 128-water build took 1.33 s, against
    // 1.21 s for the same build with sequential slabs.
    const bool may_overlap = allow_overlap && !with_D && !delta && !p.host_B && p.naux_pad >= 2 * kPadAux &&
                             !is_int8(precision);
    const double per_aux = (double)p.nao * L.ncol *
                           (esz + (with_D ? 8 : 0)) *
                           (delta ? 2 : 1) * (may_overlap ? 2 : 1);
    int64_t slab = p.host_B ? p.host_slab
                 : force_slab > 0 ? force_slab
                 : p.aux_slab > 0 ? (int64_t)align_up((size_t)p.aux_slab, kPadAux)
                                  : (int64_t)(kAutoSlabBytes / per_aux) / kPadAux * kPadAux;
    if (is_int8(precision) && !p.host_B) {   // 128 rows of int8 slices below 4 GiB (32-bit offsets)
        const int64_t ncol_e = L.ncol + (L.ncol & 1);
        const int64_t cap = ((int64_t)UINT32_MAX / (128 * kI8Slices) / ncol_e) / kPadAux * kPadAux;
        if (slab > cap) slab = cap;
        // an int8 build that needs several automatic slabs takes slabs of at
        // most 1,024 aux: on the 128-water cluster (640 orbitals) 512 / 768 /
        // 1024 / 1536 / 2048 / 3840 aux per slab measured 1.17 / 1.16 / 1.15 /
        // 1.18 / 1.28 / 1.43 s per build (the GEMM's k range per workgroup
        // grows with the slab).  A molecule that fits one slab keeps it.
        if (force_slab <= 0 && p.aux_slab <= 0 && slab < p.naux_pad && slab > kI8AutoSlab) slab = kI8AutoSlab;
    }
    if (slab < kPadAux) slab = kPadAux;
    if (slab > p.naux_pad) slab = p.naux_pad;
    L.slab = slab;
    L.nslab = (p.naux_pad + slab - 1) / slab;
    L.overlap = may_overlap && L.nslab >= 2;
    L.j_side = allow_overlap && !p.host_B;
    L.kdim = x_kdim(precision, slab, L.ncol);
    const int ntiles = delta ? L.ntile * L.ntile : L.ntile * (L.ntile + 1) / 2;
    // FP64 syrk: enough splits for 64 workgroups per CU with 64-wide tiles
    // and 16 with 128-wide ones (one workgroup fills a CU's LDS; short k
    // ranges keep a split's panels in L2).  On the 32-water cluster, 64-wide
    // tiles x 16 / 32 / 64 / 128 splits: 10.56 / 10.06 / 9.81 / 9.61 ms per
    // build; 128-wide x 8 / 16 / 32: 17.9 / 14.3 / 12.4 ms.  A split count of
    // 8 or more is rounded down to a multiple of the XCD count, so that the
    // syrk runs whole splits per XCD.
    L.nsplit_k = precision == DFJK_FP64 ? xcd_round(choose_ksplit(ntiles, L.kdim, p.num_cus, L.ktile == 64 ? 64 : L.ktile == 96 ? 32 : 16))
               : is_int8(precision) ? i8_nsplit(p.nao, L.kdim, !delta, p.num_cus)
                                              : mixed_nsplit(p.nao, L.kdim, !delta, p.num_cus);
    if (nsplit == 0 && !with_D && !delta) {   // a split count the autotuner measured for this shape
        const auto it = p.tuned_nsplit.find((int64_t)nocc * 4 + precision);
        if (it != p.tuned_nsplit.end()) nsplit = it->second;
    }
    if (nsplit > 0) {   // a batch (or the autotuner) chooses the split count
        const int64_t maxs = L.kdim / 256 > 0 ? L.kdim / 256 : 1;
        L.nsplit_k = nsplit < maxs ? nsplit : (int)maxs;
    }
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
    const size_t xb = x_bytes(precision, p.nao, L.kdim), xlo = x_lo_bytes(precision, p.nao, L.kdim);
    L.o_X = take(xb);
    L.o_Xlo = xlo ? take(xlo) : 0;
    L.o_Bfull = with_D ? take(nx * 8) : 0;
    const size_t cpad = (size_t)(p.nao + 1) * ht_ldc(L.ncol) * 8;
    L.o_Cp = take(cpad);
    L.o_Cp2 = delta ? take(cpad) : 0;
    if (L.overlap) {
        L.o_Xb = take(xb);
        L.o_Xblo = xlo ? take(xlo) : 0;
    }
    if (delta) {
        L.o_X2 = take(xb);
        L.o_X2lo = xlo ? take(xlo) : 0;
        L.o_U = take((size_t)p.nao * nocc * 8);
        L.o_W = take((size_t)p.nao * nocc * 8);
        L.o_Cr = take((size_t)p.nao * nocc * 8);
        L.o_align = take(align_work_doubles(nocc) * 8);
    }
    L.o_Kpart = take((size_t)L.nslab * L.nsplit_k * ntiles * L.ktile * L.ktile * 8);
    if (p.host_B) {   // two staging buffers for slabs of the host-resident B
        L.o_stage[0] = take((size_t)p.nf_pad * L.slab * 8);
        L.o_stage[1] = take((size_t)p.nf_pad * L.slab * 8);
    }
    L.o_Epart = take((size_t)L.ntile * (L.ntile + 1) / 2 * reduce_chunks(L.ktile) * 8);
    L.bytes = align_up(off, 256);
    return L;
}

void launch_gemm_mixed(int precision, bool lower, const void *A, const void *Alo, const void *B, const void *Blo,
                       int64_t nao, int64_t kdim, int nsplit, double *part, hipStream_t s);

// J from the resident B and the density in scratch (steps 2-4).
static void launch_j(Plan &p, const BuildLayout &L, const double *D, double *J, char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    double *dvec = reinterpret_cast<double *>(scratch + L.o_d);
    double *cpart = reinterpret_cast<double *>(scratch + L.o_cpart);
    double *cvec = reinterpret_cast<double *>(scratch + L.o_c);
    hipLaunchKernelGGL(k_gather_d, dim3((unsigned)((p.nf_pad + 255) / 256)), dim3(256), 0, s, D, nao, p.d.f_mu,
                       p.d.f_nu, p.d.f_w, p.nf, p.nf_pad, dvec);
    hipLaunchKernelGGL(k_c_partial, dim3((unsigned)((ld + 255) / 256), L.nsplit_c), dim3(256), 0, s, p.d.B, ld,
                       dvec, p.nf_pad, cpart);
    hipLaunchKernelGGL(k_c_reduce, dim3((unsigned)((ld + 255) / 256)), dim3(256), 0, s, cpart, L.nsplit_c, ld,
                       cvec);
    fill(J, nao * nao, 0.0, s);
    if (p.nf > 0)
        hipLaunchKernelGGL(k_j_rows, dim3((unsigned)((p.nf + 3) / 4)), dim3(256), 0, s, p.d.B, ld, cvec, p.d.f_mu,
                           p.d.f_nu, p.d.f_w, p.nf, nao, 0, J);
}

// The zero-padded copy of the coefficients that the half transform reads
// (k_pad_coef), in the build scratch at `off`.
static const double *pad_coef(const Plan &p, const double *C, int32_t ncol, char *scratch, size_t off, hipStream_t s)
{
    double *Cp = reinterpret_cast<double *>(scratch + off);
    const int64_t ldc = ht_ldc(ncol), n = (p.nao + 1) * ldc;
    hipLaunchKernelGGL(k_pad_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, p.nao, ncol, (int32_t)ldc,
                       Cp);
    return Cp;
}

// Half transform of one aux slab of B (rows ld apart) with padded coefficients Cp.
static HTArgs ht_args(const Plan &p, int precision, const double *B, int64_t ld, const double *Cp, int32_t ncol,
                      int64_t p_begin, int64_t plen, void *X, void *Xlo)
{
    return HTArgs{B, ld, Cp, ncol, (int32_t)ht_ldc(ncol), p.d.hk_off, p.d.hk_row, p.d.hk_nu, X, Xlo, p_begin, plen,
                  p.d.hk_order, precision == DFJK_MIXED_INT8_FAST ? kI8Slices - 1 : kI8Slices};
}

static void launch_ht(const Plan &p, int precision, const double *B, int64_t ld, const double *Cp, int32_t ncol,
                      int64_t p_begin, int64_t plen, void *X, void *Xlo, hipStream_t s)
{
    dispatch_halftrans(precision, ht_args(p, precision, B, ld, Cp, ncol, p_begin, plen, X, Xlo), p.nao, s);
}

// Steps 5-6 for every aux slab: the half transform of C1 (and of C2 for the
// increment, which contracts X(C1) with X(C2) over all tiles), then the slab's
// K contribution into its own split-K partials: lower tiles of X X^T (C route),
// X B~^T (density route, B~ the expanded tensor) or every tile of X1 X2^T.
// ncol <= L.ncol columns; slabs reuse the X buffers and the stream orders them.
static void slab_gemm(const BuildLayout &L, bool lower, const void *X, const void *Xlo, const void *Bop,
                      const void *Bop_lo, int64_t nao, int64_t kdim, double *part, hipStream_t s)
{
    if (L.precision == DFJK_FP64) {
        const int64_t ksplit = (int64_t)align_up((size_t)((kdim + L.nsplit_k - 1) / L.nsplit_k), 16);
        launch_syrk_f64(lower, static_cast<const double *>(X), static_cast<const double *>(Bop), nao, kdim, ksplit,
                        L.nsplit_k, L.ktile, part, s);
    } else if (is_int8(L.precision)) {
        launch_gemm_i8(lower, X, static_cast<const double *>(Xlo), Bop, static_cast<const double *>(Bop_lo), nao,
                       kdim, L.nsplit_k, L.precision == DFJK_MIXED_INT8_FAST, part, s);
    } else {
        launch_gemm_mixed(L.precision, lower, X, Xlo, Bop, Bop_lo, nao, kdim, L.nsplit_k, part, s);
    }
}

// The overlapped schedule of a C-route contraction: the half transform of
// slab s goes to the plan's second stream into X buffer s % 2, after the K
// GEMM that last read that buffer; the GEMM of slab s waits for it on `s`.
// Every side-stream launch is joined back into `s` by the GEMM's wait.
static bool overlap_streams(Plan &p)
{
    if (p.ht_stream) return true;
    hipEvent_t ev[5] = {};
    hipStream_t hs = nullptr;
    bool ok = true;
    for (hipEvent_t &e : ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {   // fall back to the single-stream schedule
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (hs) (void)hipStreamDestroy(hs);
        return false;
    }
    p.ev_fork = ev[0]; p.ev_ht[0] = ev[1]; p.ev_ht[1] = ev[2]; p.ev_kdone[0] = ev[3]; p.ev_kdone[1] = ev[4];
    p.ht_stream = hs;
    return true;
}

static void contract_slabs_overlapped(Plan &p, const BuildLayout &L, const double *C, int64_t ncol, char *scratch,
                                      hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    Profiler &pr = p.prof;
    void *X[2] = {scratch + L.o_X, scratch + L.o_Xb};
    void *Xlo[2] = {L.o_Xlo ? scratch + L.o_Xlo : nullptr, L.o_Xblo ? scratch + L.o_Xblo : nullptr};
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    const int ntiles = L.ntile * (L.ntile + 1) / 2;
    const size_t slab_part = (size_t)L.nsplit_k * ntiles * L.ktile * L.ktile;
    hipStream_t hs = p.ht_stream;
    const double *Cp = pad_coef(p, C, (int32_t)ncol, scratch, L.o_Cp, s);
    (void)hipEventRecord(p.ev_fork, s);
    (void)hipStreamWaitEvent(hs, p.ev_fork, 0);
    auto ht = [&](int64_t sl) {
        const int b = (int)(sl & 1);
        const int64_t pb = sl * L.slab, plen = (ld - pb < L.slab) ? ld - pb : L.slab;
        if (sl >= 2) (void)hipStreamWaitEvent(hs, p.ev_kdone[b], 0);
        pr.stream = hs;
        pr.mark(ST_HALFTRANS, true);
        launch_ht(p, L.precision, p.d.B, ld, Cp, (int32_t)ncol, pb, plen, X[b], Xlo[b], hs);
        pr.mark(ST_HALFTRANS, false);
        pr.stream = s;
        (void)hipEventRecord(p.ev_ht[b], hs);
    };
    ht(0);
    for (int64_t sl = 0; sl < L.nslab; ++sl) {
        const int b = (int)(sl & 1);
        const int64_t pb = sl * L.slab, plen = (ld - pb < L.slab) ? ld - pb : L.slab;
        if (sl + 1 < L.nslab) ht(sl + 1);
        (void)hipStreamWaitEvent(s, p.ev_ht[b], 0);
        pr.mark(ST_K, true);
        slab_gemm(L, true, X[b], Xlo[b], X[b], Xlo[b], nao, x_kdim(L.precision, plen, ncol), Kpart + sl * slab_part,
                  s);
        pr.mark(ST_K, false);
        (void)hipEventRecord(p.ev_kdone[b], s);
    }
}

static void contract_slabs(Plan &p, const BuildLayout &L, const double *C1, const double *C2, int64_t ncol,
                           char *scratch, hipStream_t s)
{
    if (L.overlap && C2 == nullptr && overlap_streams(p)) {
        contract_slabs_overlapped(p, L, C1, ncol, scratch, s);
        return;
    }
    const int64_t nao = p.nao, ld = p.naux_pad;
    Profiler &pr = p.prof;
    void *X = scratch + L.o_X;
    void *Xlo = L.o_Xlo ? scratch + L.o_Xlo : nullptr;
    double *Bt = L.o_Bfull ? reinterpret_cast<double *>(scratch + L.o_Bfull) : nullptr;
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    const bool lower = !L.delta;
    const int ntiles = lower ? L.ntile * (L.ntile + 1) / 2 : L.ntile * L.ntile;
    const size_t slab_part = (size_t)L.nsplit_k * ntiles * L.ktile * L.ktile;
    void *X2 = L.delta ? scratch + L.o_X2 : nullptr;
    void *X2lo = L.o_X2lo ? scratch + L.o_X2lo : nullptr;
    const double *Cp1 = pad_coef(p, C1, (int32_t)ncol, scratch, L.o_Cp, s);
    const double *Cp2 = L.delta ? pad_coef(p, C2, (int32_t)ncol, scratch, L.o_Cp2, s) : nullptr;
    for (int64_t sl = 0; sl < L.nslab; ++sl) {
        const int64_t pb = sl * L.slab, plen = (ld - pb < L.slab) ? ld - pb : L.slab;
        const int64_t kdim = x_kdim(L.precision, plen, ncol);
        pr.mark(ST_HALFTRANS, true);
        launch_ht(p, L.precision, p.d.B, ld, Cp1, (int32_t)ncol, pb, plen, X, Xlo, s);
        if (L.norms)
            launch_i8_norms(X, static_cast<const double *>(Xlo), nao, kdim, reinterpret_cast<double *>(scratch + L.o_norms),
                            s);
        if (L.delta)
            launch_ht(p, L.precision, p.d.B, ld, Cp2, (int32_t)ncol, pb, plen, X2, X2lo, s);
        else if (L.with_D)
            hipLaunchKernelGGL(k_expand_B, dim3((unsigned)((plen + 255) / 256), (unsigned)nao), dim3(256), 0, s,
                               p.d.B, ld, p.d.hk_off, p.d.hk_row, p.d.hk_nu, nao, pb, plen, Bt);
        pr.mark(ST_HALFTRANS, false);
        pr.mark(ST_K, true);
        const void *Bop = L.delta ? (const void *)X2 : (L.with_D ? (const void *)Bt : (const void *)X);
        const void *Bop_lo = L.delta ? (const void *)X2lo : Xlo;
        slab_gemm(L, lower, X, Xlo, Bop, Bop_lo, nao, kdim, Kpart + sl * slab_part, s);
        pr.mark(ST_K, false);
    }
}

// The plan's side stream and its fork / join events (created on first use;
// false if HIP refuses, and the caller then runs the work in turn on its
// own stream).  A build runs J there; a setup runs the integrals there.
bool side_stream(Plan &p)
{
    if (p.j_stream) return true;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t js = nullptr;
    bool ok = hipEventCreateWithFlags(&a, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&js, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (js) (void)hipStreamDestroy(js);
        return false;
    }
    p.ev_jfork = a; p.ev_jdone = b; p.j_stream = js;
    return true;
}

void launch_build(Plan &p, const BuildLayout &L, const double *C, const double *Din, double *J, double *K,
                  double *E, char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    double *D = reinterpret_cast<double *>(scratch + L.o_D);
    double *cvec = reinterpret_cast<double *>(scratch + L.o_c);
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    double *Epart = reinterpret_cast<double *>(scratch + L.o_Epart);
    Profiler &pr = p.prof;
    pr.stream = s;
    pr.mark(ST_BUILD, true);

    // 1. density
    pr.mark(ST_DENSITY, true);
    if (!L.with_D) {
        dim3 grid((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16));
        hipLaunchKernelGGL(k_density, grid, dim3(256), 0, s, C, nao, (int32_t)L.ncol, 2.0, D);
    } else {
        (void)hipMemcpyAsync(D, Din, (size_t)nao * nao * 8, hipMemcpyDeviceToDevice, s);
    }
    if (L.delta) {   // U, W from C rotated onto C0 (D is unchanged by the rotation)
        double *Cr = reinterpret_cast<double *>(scratch + L.o_Cr);
        launch_align(C, L.C0, nao, (int32_t)L.ncol, reinterpret_cast<double *>(scratch + L.o_align), Cr, s);
        hipLaunchKernelGGL(k_uw, dim3((unsigned)((nao * L.ncol + 255) / 256)), dim3(256), 0, s, Cr, L.C0, nao,
                           (int32_t)L.ncol, reinterpret_cast<double *>(scratch + L.o_U),
                           reinterpret_cast<double *>(scratch + L.o_W));
    }
    pr.mark(ST_DENSITY, false);
    // 2-4. J (always FP64).  J streams B through HBM (bound there) while the
    // half transform and K are bound by the FP64 MFMA pipes, so J runs on a
    // side stream beside them and is joined before the energies: it reads
    // D and B and writes only J and its own scratch (d, c partials, c).
    const bool jside = L.j_side && side_stream(p);
    hipStream_t js = jside ? p.j_stream : s;
    if (jside) {
        (void)hipEventRecord(p.ev_jfork, s);
        (void)hipStreamWaitEvent(js, p.ev_jfork, 0);
        pr.stream = js;
    }
    pr.mark(ST_J, true);
    launch_j(p, L, D, J, scratch, js);
    pr.mark(ST_J, false);
    if (jside) {
        (void)hipEventRecord(p.ev_jdone, js);
        pr.stream = s;
    }
    // 5-6. per aux slab: half transform(s) and the slab's K contribution
    if (!L.delta)
        contract_slabs(p, L, L.with_D ? Din : C, nullptr, L.ncol, scratch, s);
    else
        contract_slabs(p, L, reinterpret_cast<double *>(scratch + L.o_U),
                       reinterpret_cast<double *>(scratch + L.o_W), L.ncol, scratch, s);
    // 7. split-K sum, mirror, energies (after J: the energies read c)
    if (jside) (void)hipStreamWaitEvent(s, p.ev_jdone, 0);
    pr.mark(ST_KREDUCE, true);
    const int nlower = L.ntile * (L.ntile + 1) / 2;
    const int64_t nep = (int64_t)nlower * (L.delta ? kTileK / 16 : reduce_chunks(L.ktile));   // energy partials
    if (L.delta)
        hipLaunchKernelGGL(k_k_reduce_delta, dim3(nlower, kTileK / 16), dim3(256), 0, s, Kpart,
                           (int)(L.nslab * L.nsplit_k),
                           L.ntile, nao, L.K0, D, K, Epart);
    else
        hipLaunchKernelGGL(k_k_reduce, dim3(nlower, reduce_chunks(L.ktile)), dim3(256), 0, s, Kpart,
                           (int)(L.nslab * L.nsplit_k), L.ntile, L.ktile, nao, L.with_D ? 1.0 : 2.0, D, K, Epart);
    hipLaunchKernelGGL(k_energies, dim3(1), dim3(256), 0, s, cvec, ld, Epart, nep, -0.25, E);
    pr.mark(ST_KREDUCE, false);
    pr.mark(ST_BUILD, false);
}

BuildLayout build_layout_uks(const Plan &p, int32_t nocc_a, int32_t nocc_b, int32_t precision)
{
    BuildLayout L = build_layout(p, nocc_a > nocc_b ? nocc_a : nocc_b, precision, false);
    L.uks = true;
    L.nocc_a = nocc_a;
    L.nocc_b = nocc_b;
    size_t off = L.bytes;
    auto take = [&](size_t bytes) {
        off = align_up(off, 256);
        const size_t o = off;
        off += bytes;
        return o;
    };
    L.o_Da = take((size_t)p.nao * p.nao * 8);
    L.o_Db = take((size_t)p.nao * p.nao * 8);
    L.o_Epart = take((size_t)2 * L.ntile * (L.ntile + 1) / 2 * reduce_chunks(L.ktile) * 8);   // one block per spin
    L.bytes = align_up(off, 256);
    return L;
}

// Open-shell build: D_s = C_s C_s^T for s = alpha, beta; J from D = D_a + D_b;
// K_s = sum_P B_P D_s B_P = X_s X_s^T; E_J = 1/2 Tr D J = 1/2 sum_P c_P^2,
// E_K = -1/2 (Tr D_a K_a + Tr D_b K_b).
void launch_build_uks(Plan &p, const BuildLayout &L, const double *Ca, const double *Cb, double *J, double *Ka,
                      double *Kb, double *E, char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    double *D = reinterpret_cast<double *>(scratch + L.o_D);
    double *Ds[2] = {reinterpret_cast<double *>(scratch + L.o_Da), reinterpret_cast<double *>(scratch + L.o_Db)};
    const double *Cs[2] = {Ca, Cb};
    double *Ks[2] = {Ka, Kb};
    const int32_t nocc[2] = {L.nocc_a, L.nocc_b};
    double *cvec = reinterpret_cast<double *>(scratch + L.o_c);
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    double *Epart = reinterpret_cast<double *>(scratch + L.o_Epart);
    const int nlower = L.ntile * (L.ntile + 1) / 2;
    const int64_t nep = (int64_t)nlower * reduce_chunks(L.ktile);
    Profiler &pr = p.prof;
    pr.stream = s;

    pr.mark(ST_DENSITY, true);
    const dim3 grid((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16));
    for (int sp = 0; sp < 2; ++sp) {
        if (nocc[sp] > 0) hipLaunchKernelGGL(k_density, grid, dim3(256), 0, s, Cs[sp], nao, nocc[sp], 1.0, Ds[sp]);
        else fill(Ds[sp], nao * nao, 0.0, s);
    }
    hipLaunchKernelGGL(k_add, dim3((unsigned)((nao * nao + 255) / 256)), dim3(256), 0, s, Ds[0], Ds[1], nao * nao, D);
    pr.mark(ST_DENSITY, false);
    pr.mark(ST_J, true);
    launch_j(p, L, D, J, scratch, s);
    pr.mark(ST_J, false);
    for (int sp = 0; sp < 2; ++sp) {
        if (nocc[sp] == 0) {
            fill(Ks[sp], nao * nao, 0.0, s);
            fill(Epart + sp * nep, nep, 0.0, s);
            continue;
        }
        contract_slabs(p, L, Cs[sp], nullptr, nocc[sp], scratch, s);
        pr.mark(ST_KREDUCE, true);
        hipLaunchKernelGGL(k_k_reduce, dim3(nlower, reduce_chunks(L.ktile)), dim3(256), 0, s, Kpart,
                           (int)(L.nslab * L.nsplit_k), L.ntile, L.ktile, nao, 1.0, Ds[sp], Ks[sp], Epart + sp * nep);
        pr.mark(ST_KREDUCE, false);
    }
    pr.mark(ST_KREDUCE, true);
    hipLaunchKernelGGL(k_energies, dim3(1), dim3(256), 0, s, cvec, ld, Epart, 2 * nep, -0.5, E);
    pr.mark(ST_KREDUCE, false);
}

// Split count shared by the molecules of a batch: enough workgroups over all
// their lower K tiles to fill one round of the chip.
int batch_nsplit(const Plan *const *plans, int n)
{
    int tiles = 0, cus = 256;
    for (int i = 0; i < n; ++i) {
        const int nt = (int)((plans[i]->nao + kTileK - 1) / kTileK);
        tiles += nt * (nt + 1) / 2;
        cus = plans[i]->num_cus;
    }
    return choose_ksplit(tiles > 0 ? tiles : 1, (int64_t)1 << 40, cus);
}

// A batch of closed-shell builds on one stream.  Per molecule: density, J and
// the half transform; then one grouped FP64 K launch over every molecule
// whose X fits one slab, one grouped split-K reduction and one grouped energy
// launch.  Mixed precision and multi-slab molecules contract on their own.
void launch_build_batch(int n, Plan *const *plans, const BuildLayout *Ls, const double *const *C, double *const *J,
                        double *const *K, double *const *E, char *const *scratch, hipStream_t s)
{
    std::vector<Plan *> joins;
    std::vector<PreArgs> pre;
    std::vector<std::pair<HTArgs, int64_t>> hts, hts8;   // arguments and AO count of each grouped half transform
    std::vector<const void *> i8x;                        // grouped int8 K: slices, scales, sizes, splits, partials
    std::vector<const double *> i8s;
    std::vector<int64_t> i8m, i8k;
    std::vector<int> i8n;
    std::vector<double *> i8p;
    bool i8fast = false;
    std::vector<const double *> kx;
    std::vector<double *> kp;
    std::vector<int64_t> km, kk, ks;
    std::vector<int> ns, kt;
    for (int i = 0; i < n; ++i) {
        Plan &p = *plans[i];
        const BuildLayout &L = Ls[i];
        char *sc = scratch[i];
        const int64_t nao = p.nao;
        double *D = reinterpret_cast<double *>(sc + L.o_D);
        if (L.nslab == 1 && (L.precision == DFJK_FP64 || is_int8(L.precision))) {
            // density, padded coefficients and J in the shared launches of
            // launch_pre_groups, the half transform and K grouped after them
            PreArgs a{};
            a.C = C[i]; a.D = D; a.J = J[i];
            a.Cp = reinterpret_cast<double *>(sc + L.o_Cp);
            a.f_mu = p.d.f_mu; a.f_nu = p.d.f_nu; a.f_w = p.d.f_w; a.B = p.d.B;
            a.dvec = reinterpret_cast<double *>(sc + L.o_d);
            a.cpart = reinterpret_cast<double *>(sc + L.o_cpart);
            a.cvec = reinterpret_cast<double *>(sc + L.o_c);
            a.nao = nao; a.nf = p.nf; a.nf_pad = p.nf_pad; a.ld = p.naux_pad;
            a.nocc = (int32_t)L.ncol; a.ldc = (int32_t)ht_ldc(L.ncol); a.nsplit_c = L.nsplit_c;
            pre.push_back(a);
            if (is_int8(L.precision)) {
                void *Xlo = sc + L.o_Xlo;   // block scales
                hts8.emplace_back(ht_args(p, L.precision, p.d.B, p.naux_pad, a.Cp, (int32_t)L.ncol, 0, p.naux_pad,
                                          sc + L.o_X, Xlo),
                                  nao);
                i8x.push_back(sc + L.o_X);
                i8s.push_back(static_cast<const double *>(Xlo));
                i8m.push_back(nao);
                i8k.push_back(x_kdim(L.precision, p.naux_pad, L.ncol));
                i8n.push_back(L.nsplit_k);
                i8p.push_back(reinterpret_cast<double *>(sc + L.o_Kpart));
                i8fast = L.precision == DFJK_MIXED_INT8_FAST;
                continue;
            }
            hts.emplace_back(ht_args(p, DFJK_FP64, p.d.B, p.naux_pad, a.Cp, (int32_t)L.ncol, 0, p.naux_pad,
                                     sc + L.o_X, nullptr),
                             nao);
            kx.push_back(reinterpret_cast<const double *>(sc + L.o_X));
            km.push_back(nao);
            kk.push_back(L.kdim);
            ks.push_back((int64_t)align_up((size_t)((L.kdim + L.nsplit_k - 1) / L.nsplit_k), 16));
            ns.push_back(L.nsplit_k);
            kt.push_back(L.ktile);
            kp.push_back(reinterpret_cast<double *>(sc + L.o_Kpart));
            continue;
        }
        p.prof.stream = s;
        p.prof.mark(ST_DENSITY, true);
        hipLaunchKernelGGL(k_density, dim3((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16)), dim3(256), 0,
                           s, C[i], nao, (int32_t)L.ncol, 2.0, D);
        p.prof.mark(ST_DENSITY, false);
        // J on the plan's side stream beside the other molecules' work,
        // joined before the energies (the only later step that reads c)
        hipStream_t js = s;
        if (side_stream(p)) {
            (void)hipEventRecord(p.ev_jfork, s);
            (void)hipStreamWaitEvent(p.j_stream, p.ev_jfork, 0);
            js = p.j_stream;
            joins.push_back(&p);
        }
        p.prof.stream = js;
        p.prof.mark(ST_J, true);
        launch_j(p, L, D, J[i], sc, js);
        p.prof.mark(ST_J, false);
        p.prof.stream = s;
        if (js != s) (void)hipEventRecord(p.ev_jdone, js);
        contract_slabs(p, L, C[i], nullptr, L.ncol, sc, s);
    }
    launch_pre_groups(pre, s);
    // the half transforms of the one-slab molecules, grouped by output and fragment count
    launch_halftrans_groups<OUT_F64>(hts, s);
    launch_halftrans_groups<OUT_I8>(hts8, s);
    if (!i8x.empty())
        launch_gemm_i8_group(i8fast, (int)i8x.size(), i8x.data(), i8s.data(), i8m.data(), i8k.data(), i8n.data(),
                             i8p.data(), s);
    for (int T : {64, 96, 128}) {   // one grouped syrk per tile width
        std::vector<const double *> gx;
        std::vector<double *> gp;
        std::vector<int64_t> gm, gk, gs;
        std::vector<int> gn;
        for (size_t i = 0; i < kx.size(); ++i)
            if (kt[i] == T) {
                gx.push_back(kx[i]); gp.push_back(kp[i]); gm.push_back(km[i]); gk.push_back(kk[i]);
                gs.push_back(ks[i]); gn.push_back(ns[i]);
            }
        if (!gx.empty())
            launch_syrk_f64_group(T, (int)gx.size(), gx.data(), gm.data(), gk.data(), gs.data(), gn.data(),
                                  gp.data(), s);
    }
    for (int first = 0; first < n; first += kReduceGroupMax) {
        ReduceGroup grp{};
        int total = 0;
        for (int i = first; i < n && grp.n < kReduceGroupMax; ++i) {
            const BuildLayout &L = Ls[i];
            const int q = grp.n++;
            grp.blk_start[q] = total;
            grp.nsplit[q] = (int32_t)(L.nslab * L.nsplit_k);
            grp.ntm[q] = L.ntile;
            grp.T[q] = L.ktile;
            grp.nao[q] = L.nao;
            grp.part[q] = reinterpret_cast<const double *>(scratch[i] + L.o_Kpart);
            grp.D[q] = reinterpret_cast<const double *>(scratch[i] + L.o_D);
            grp.K[q] = K[i];
            grp.Epart[q] = reinterpret_cast<double *>(scratch[i] + L.o_Epart);
            total += L.ntile * (L.ntile + 1) / 2;
        }
        grp.blk_start[grp.n] = total;
        hipLaunchKernelGGL(k_k_reduce_grouped, dim3(total, reduce_chunks(kTileK)), dim3(256), 0, s, grp, 2.0);
    }
    for (Plan *p : joins) (void)hipStreamWaitEvent(s, p->ev_jdone, 0);
    for (int first = 0; first < n; first += kEnergyGroupMax) {
        EnergyGroup grp{};
        int m = 0;
        for (int i = first; i < n && m < kEnergyGroupMax; ++i, ++m) {
            const BuildLayout &L = Ls[i];
            grp.c[m] = reinterpret_cast<const double *>(scratch[i] + L.o_c);
            grp.naux[m] = L.naux_pad;
            grp.Epart[m] = reinterpret_cast<const double *>(scratch[i] + L.o_Epart);
            grp.nEpart[m] = (int64_t)L.ntile * (L.ntile + 1) / 2 * reduce_chunks(L.ktile);
            grp.E[m] = E[i];
        }
        hipLaunchKernelGGL(k_energies_grouped, dim3(m), dim3(256), 0, s, grp, -0.25);
    }
}

// Closed-shell build from a host-resident B (paper Section 2.1: integrals in
// host memory, moved to the GPU asynchronously).  The host copy is slab-major
// ([slab][f][plen], the slab width fixed when B was offloaded); each slab is
// copied into one of two staging buffers on the plan's copy stream while the
// previous slab is consumed on `s`: c for the slab's aux functions, its
// contribution to J, the half transform and the slab's K partial tiles.
// Events order the two streams: the copy into a buffer waits for the compute
// that last read it; the compute waits for its copy.
void launch_build_hostB(Plan &p, const BuildLayout &L, const double *C, double *J, double *K, double *E,
                        char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao, ld = p.naux_pad;
    double *D = reinterpret_cast<double *>(scratch + L.o_D);
    double *dvec = reinterpret_cast<double *>(scratch + L.o_d);
    double *cpart = reinterpret_cast<double *>(scratch + L.o_cpart);
    double *cvec = reinterpret_cast<double *>(scratch + L.o_c);
    double *Kpart = reinterpret_cast<double *>(scratch + L.o_Kpart);
    double *Epart = reinterpret_cast<double *>(scratch + L.o_Epart);
    double *stage[2] = {reinterpret_cast<double *>(scratch + L.o_stage[0]),
                        reinterpret_cast<double *>(scratch + L.o_stage[1])};
    void *X = scratch + L.o_X;
    void *Xlo = L.o_Xlo ? scratch + L.o_Xlo : nullptr;
    const int ntiles = L.ntile * (L.ntile + 1) / 2;
    const size_t slab_part = (size_t)L.nsplit_k * ntiles * L.ktile * L.ktile;
    Profiler &pr = p.prof;
    pr.stream = s;
    hipStream_t cs = p.copy_stream;

    auto copy_slab = [&](int64_t sl) {
        const int b = (int)(sl & 1);
        const int64_t pb = sl * L.slab, plen = (ld - pb < L.slab) ? ld - pb : L.slab;
        (void)hipStreamWaitEvent(cs, p.ev_free[b], 0);
        (void)hipMemcpyAsync(stage[b], p.hB + (size_t)p.nf_pad * pb, (size_t)p.nf_pad * plen * 8,
                             hipMemcpyHostToDevice, cs);
        (void)hipEventRecord(p.ev_ready[b], cs);
    };
    // the copy stream starts after everything already queued on s
    (void)hipEventRecord(p.ev_start, s);
    (void)hipStreamWaitEvent(cs, p.ev_start, 0);
    copy_slab(0);
    if (L.nslab > 1) copy_slab(1);

    pr.mark(ST_DENSITY, true);
    hipLaunchKernelGGL(k_density, dim3((unsigned)((nao + 15) / 16), (unsigned)((nao + 15) / 16)), dim3(256), 0, s, C,
                       nao, (int32_t)L.ncol, 2.0, D);
    pr.mark(ST_DENSITY, false);
    hipLaunchKernelGGL(k_gather_d, dim3((unsigned)((p.nf_pad + 255) / 256)), dim3(256), 0, s, D, nao, p.d.f_mu,
                       p.d.f_nu, p.d.f_w, p.nf, p.nf_pad, dvec);
    fill(J, nao * nao, 0.0, s);
    const double *Cp = pad_coef(p, C, (int32_t)L.ncol, scratch, L.o_Cp, s);
    for (int64_t sl = 0; sl < L.nslab; ++sl) {
        const int b = (int)(sl & 1);
        const int64_t pb = sl * L.slab, plen = (ld - pb < L.slab) ? ld - pb : L.slab;
        (void)hipStreamWaitEvent(s, p.ev_ready[b], 0);
        pr.mark(ST_J, true);
        hipLaunchKernelGGL(k_c_partial, dim3((unsigned)((plen + 255) / 256), L.nsplit_c), dim3(256), 0, s, stage[b],
                           plen, dvec, p.nf_pad, cpart);
        hipLaunchKernelGGL(k_c_reduce, dim3((unsigned)((plen + 255) / 256)), dim3(256), 0, s, cpart, L.nsplit_c,
                           plen, cvec + pb);
        if (p.nf > 0)
            hipLaunchKernelGGL(k_j_rows, dim3((unsigned)((p.nf + 3) / 4)), dim3(256), 0, s, stage[b], plen, cvec + pb,
                               p.d.f_mu, p.d.f_nu, p.d.f_w, p.nf, nao, 1, J);
        pr.mark(ST_J, false);
        pr.mark(ST_HALFTRANS, true);
        launch_ht(p, L.precision, stage[b], plen, Cp, (int32_t)L.ncol, 0, plen, X, Xlo, s);
        if (L.norms)
            launch_i8_norms(X, static_cast<const double *>(Xlo), nao, x_kdim(L.precision, plen, L.ncol),
                            reinterpret_cast<double *>(scratch + L.o_norms), s);
        pr.mark(ST_HALFTRANS, false);
        (void)hipEventRecord(p.ev_free[b], s);      // the staging buffer is read
        if (sl + 2 < L.nslab) copy_slab(sl + 2);
        pr.mark(ST_K, true);
        const int64_t kdim = x_kdim(L.precision, plen, L.ncol);
        slab_gemm(L, true, X, Xlo, X, Xlo, nao, kdim, Kpart + sl * slab_part, s);
        pr.mark(ST_K, false);
    }
    pr.mark(ST_KREDUCE, true);
    const int nlower = L.ntile * (L.ntile + 1) / 2;
    hipLaunchKernelGGL(k_k_reduce, dim3(nlower, reduce_chunks(L.ktile)), dim3(256), 0, s, Kpart, (int)(L.nslab * L.nsplit_k),
                       L.ntile, L.ktile, nao, 2.0, D, K, Epart);
    hipLaunchKernelGGL(k_energies, dim3(1), dim3(256), 0, s, cvec, ld, Epart, (int64_t)nlower * reduce_chunks(L.ktile), -0.25,
                       E);
    pr.mark(ST_KREDUCE, false);
    pr.mark(ST_BUILD, false);
}

}  // namespace dfjk
