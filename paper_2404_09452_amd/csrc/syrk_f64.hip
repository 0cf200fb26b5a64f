// FP64 K contraction with operands moved by LDS DMA: the split-K partial
// tiles of C = A B^T (A, B: rows of the half-transformed tensor, k
// contiguous), lower tiles only for K = X X^T or every tile for the
// increment's X1 X2^T.  Same partial layout and the same order of the FP64
// MFMA accumulation per element as the register-staged tile GEMM
// (gemm_f64.h): chunks of 16 k in ascending order, four k per MFMA step.
//
// Workgroup: one T x T tile of one k split, WGM x WGN waves (T = 128: 4 x 2
// waves of 32 x 64; T = 96: 2 x 2 waves of 48 x 48; T = 64: 2 x 2 waves of
// 32 x 32), v_mfma_f64_16x16x4f64
// (lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator r of lane l
// is D[l/16 + 4r][l%16]).
//
// Operands go from global memory straight into LDS
// (global_load_lds_dwordx4: 16 bytes per lane, the lanes of one instruction
// filling 1 KB in lane order) through a ring of three chunk buffers, two
// chunks in flight while the MFMAs use the third; one barrier per chunk.
// One instruction brings 8 rows x 16 k of one operand; inside it lane l
// holds row r = l/8 and k pair p = (l%8) xor (r%8), so the k pair of a row
// is stored at slot p xor (r%8): the 64 lanes of a fragment read (16 rows x
// 4 k) then fall on every 16-byte bank group twice, the minimum for 512
// bytes.  Rows past M read row M-1; their products reach only outputs the
// reduction drops.
#include "dfjk_internal.h"

namespace dfjk {

namespace {

constexpr int kSyrkKC = 16;          // k per chunk (three chunk buffers)

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct SyrkArgs {
    const double *A, *B;             // [M][ld], [N][ld] rows, k contiguous
    int64_t ld, M, N;
    int64_t kdim, ksplit;            // ksplit: a multiple of kSyrkKC
    int ntm, ntn;                    // tiles along M and N
    int lower;                       // 1: tiles with tn <= tm (K = X X^T), else every tile
    int tri_k;                       // 1: B(n, k) = 0 for k > n, so a tile stops at its last column
    int nsplit;
    double *partial;                 // [split][tile][T][T], or
    double *C;                       // C[m][n] (ldc) when partial is null
    int64_t ldc;
};

// s_waitcnt immediates (gfx9: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt
// 11:8; a field at its maximum does not wait)
template <int N> constexpr int wait_vm() { return (N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8); }

// Workgroup `blk` of a launch over g (ntiles x nsplit workgroups).
template <int T, int WGM, int WGN>
__device__ __forceinline__ void syrk_tile(SyrkArgs g, unsigned blk)
{
    constexpr int NW = WGM * WGN;
    constexpr int WTM = T / WGM, WTN = T / WGN, MB = WTM / 16, NB = WTN / 16;
    constexpr int OPD = T * kSyrkKC;                 // doubles of one operand's chunk
    constexpr int NI = 2 * T / 8;                    // DMA instructions per chunk (8 rows each)
    constexpr int NIW = NI / NW;                     // per wave
    static_assert(NIW * NW == NI && NIW <= 15, "DMA instructions must spread evenly over the waves");
    __shared__ __attribute__((aligned(1024))) double s0[2 * OPD];
    __shared__ __attribute__((aligned(1024))) double s1[2 * OPD];
    __shared__ __attribute__((aligned(1024))) double s2[2 * OPD];

    const int ntiles = g.lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntn;
    // workgroup -> (split, tile), 1-D grid.  With a split count that is a
    // multiple of the XCD count, XCD x (workgroups go round-robin over the
    // XCDs) runs whole splits x, x + 8, ...: the tiles of one k range share
    // their panels in one L2 instead of every L2 fetching every panel.
    int tile, split;
    if (g.nsplit % kXcds == 0) {
        const int xcd = blk % kXcds, local = blk / kXcds;
        split = xcd + kXcds * (local / ntiles);
        tile = local % ntiles;
    } else {
        split = blk / ntiles;
        tile = blk % ntiles;
    }
    int tm, tn;
    if (g.lower) {
        int r = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
        while (r * (r + 1) / 2 > tile) --r;
        while ((r + 1) * (r + 2) / 2 <= tile) ++r;
        tm = r;
        tn = tile - r * (r + 1) / 2;
    } else {
        tm = tile % g.ntm;
        tn = tile / g.ntm;
        if (g.tri_k) tn = g.ntn - 1 - tn;   // the longest k ranges first
    }
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WGN, wn = wave % WGN;
    const int64_t kb = (int64_t)split * g.ksplit;
    int64_t ke = min(kb + g.ksplit, g.kdim);
    if (g.tri_k) ke = min(ke, (int64_t)(tn + 1) * T);
    const int nch = (int)((ke - kb) / kSyrkKC);

    // this lane's global offset (doubles, relative to the chunk's k0) for each
    // DMA instruction of its wave
    int64_t goff[NIW];
#pragma unroll
    for (int q = 0; q < NIW; ++q) {
        const int ins = wave * NIW + q;
        const bool isA = ins < NI / 2;
        const int r = (ins % (NI / 2)) * 8 + lane / 8;
        const int p = (lane % 8) ^ (r % 8);
        const int64_t row = isA ? min((int64_t)tm * T + r, g.M - 1) : min((int64_t)tn * T + r, g.N - 1);
        goff[q] = row * g.ld + 2 * p;
    }
    auto dma = [&](int c, double *buf) {
        const int64_t k0 = kb + (int64_t)min(c, nch - 1) * kSyrkKC;   // past the end: the last chunk again
#pragma unroll
        for (int q = 0; q < NIW; ++q) {
            const int ins = wave * NIW + q;
            const bool isA = ins < NI / 2;
            const double *src = (isA ? g.A : g.B) + goff[q] + k0;
            double *dst = buf + (isA ? 0 : OPD) + (ins % (NI / 2)) * 8 * kSyrkKC;
            __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)dst, 16,
                                             0, 0);
        }
    };

    f64x4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    // fragment read offset of step ks: row (lane % 16) of the fragment, k
    // 4 ks + lane / 16 -> pair 2 ks + lane / 32 (swizzled), parity (lane / 16) % 2
    int roff[kSyrkKC / 4];
#pragma unroll
    for (int ks = 0; ks < kSyrkKC / 4; ++ks)
        roff[ks] = (lane & 15) * kSyrkKC + (((2 * ks + (lane >> 5)) ^ (lane & 7)) << 1) + ((lane >> 4) & 1);

    auto mfma = [&](const double *buf) {
        const double *as = buf + wm * WTM * kSyrkKC;
        const double *bs = buf + OPD + wn * WTN * kSyrkKC;
#pragma unroll
        for (int ks = 0; ks < kSyrkKC / 4; ++ks) {
            double a[MB], b[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) a[i] = as[i * 16 * kSyrkKC + roff[ks]];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = bs[j * 16 * kSyrkKC + roff[ks]];
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
    // chunk c: its DMA has landed for this wave once only the NIW loads of
    // chunk c + 1 are outstanding; the barrier makes that true for every
    // wave and tells that chunk c - 1's buffer is read; then the DMA of
    // chunk c + 2 goes into that buffer and the MFMAs run on chunk c
    auto step = [&](int c, const double *cur, double *nxt2) {
        __builtin_amdgcn_s_waitcnt(wait_vm<NIW>());
        __builtin_amdgcn_s_barrier();
        dma(c + 2, nxt2);
        __builtin_amdgcn_sched_barrier(0);
        mfma(cur);
        __builtin_amdgcn_sched_barrier(0);
    };

    if (nch > 0) {
        dma(0, s0);
        dma(1, s1);
        int c = 0;
        for (; c + 3 <= nch; c += 3) {   // whole rounds of the three buffers
            step(c, s0, s2);
            step(c + 1, s1, s0);
            step(c + 2, s2, s1);
        }
        if (c < nch) step(c, s0, s2);
        if (c + 1 < nch) step(c + 1, s1, s0);
        __builtin_amdgcn_s_waitcnt(wait_vm<0>());   // no DMA into LDS outlives the workgroup
    }

    if (g.partial) {
        double *dst = g.partial + ((int64_t)split * ntiles + tile) * (int64_t)(T * T);
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * WTM + i * 16 + (lane >> 4) + 4 * r;
                    const int col = wn * WTN + j * 16 + (lane & 15);
                    dst[row * T + col] = acc[i][j][r];
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = (int64_t)tm * T + wm * WTM + i * 16 + (lane >> 4) + 4 * r;
                const int64_t n = (int64_t)tn * T + wn * WTN + j * 16 + (lane & 15);
                if (m < g.M && n < g.N) g.C[m * g.ldc + n] = acc[i][j][r];
            }
}

template <int T, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(T == 64 ? 3 : 2)))
void k_syrk_f64(SyrkArgs g)
{
    syrk_tile<T, WGM, WGN>(g, blockIdx.x);
}

// The K syrk of several molecules in one launch (batches of small
// molecules): workgroup b runs workgroup b - blk_start[m] of molecule m's own
// launch, descriptors by value (no device table, so the launch can be
// captured).  Each molecule's partial tiles are those of its own launch.
constexpr int kSyrkGroupMax = 16;
struct SyrkGroup {
    int32_t n;
    uint32_t blk_start[kSyrkGroupMax + 1];
    SyrkArgs g[kSyrkGroupMax];
};
static_assert(sizeof(SyrkGroup) <= 4096, "kernel arguments are limited to 4 KB");

template <int T, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(T == 64 ? 3 : 2)))
void k_syrk_f64_group(SyrkGroup grp)
{
    int m = 0;
    while (m + 1 < grp.n && blockIdx.x >= grp.blk_start[m + 1]) ++m;
    syrk_tile<T, WGM, WGN>(grp.g[m], blockIdx.x - grp.blk_start[m]);
}

}  // namespace

// Split-K partial tiles of A B^T (A = B for the lower-tile syrk): M rows of
// kdim, nsplit splits of ksplit (a multiple of 16), tiles of T (64, 96 or 128).
void launch_syrk_f64(bool lower, const double *A, const double *B, int64_t M, int64_t kdim, int64_t ksplit,
                     int nsplit, int T, double *partial, hipStream_t s)
{
    SyrkArgs g{};
    g.A = A; g.B = B; g.ld = kdim; g.M = M; g.N = M; g.kdim = kdim; g.ksplit = ksplit;
    g.ntm = g.ntn = (int)((M + T - 1) / T);
    g.lower = lower ? 1 : 0;
    g.nsplit = nsplit;
    g.partial = partial;
    const int ntiles = lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntn;
    if (ntiles <= 0 || nsplit <= 0) return;
    const unsigned nwg = (unsigned)(ntiles * nsplit);
    if (T == 128)
        hipLaunchKernelGGL((k_syrk_f64<128, 4, 2>), dim3(nwg), dim3(512), 0, s, g);
    else if (T == 96)
        hipLaunchKernelGGL((k_syrk_f64<96, 2, 2>), dim3(nwg), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_syrk_f64<64, 2, 2>), dim3(nwg), dim3(256), 0, s, g);
}

// Lower-tile syrk partials of several molecules on T-wide tiles (64, 96 or
// 128), up to kSyrkGroupMax per launch: molecule i has M[i] rows of X (A[i], kdim[i]
// long), nsplit[i] splits of ksplit[i] (a multiple of 16) and its partials
// at partial[i], laid out as launch_syrk_f64 lays them out.
void launch_syrk_f64_group(int T, int n, const double *const *A, const int64_t *M, const int64_t *kdim,
                           const int64_t *ksplit, const int *nsplit, double *const *partial, hipStream_t s)
{
    SyrkGroup grp{};
    int64_t total = 0;
    auto flush = [&]() {
        if (grp.n == 0) return;
        grp.blk_start[grp.n] = (uint32_t)total;
        if (T == 128)
            hipLaunchKernelGGL((k_syrk_f64_group<128, 4, 2>), dim3((unsigned)total), dim3(512), 0, s, grp);
        else if (T == 96)
            hipLaunchKernelGGL((k_syrk_f64_group<96, 2, 2>), dim3((unsigned)total), dim3(256), 0, s, grp);
        else
            hipLaunchKernelGGL((k_syrk_f64_group<64, 2, 2>), dim3((unsigned)total), dim3(256), 0, s, grp);
        grp = SyrkGroup{};
        total = 0;
    };
    for (int i = 0; i < n; ++i) {
        SyrkArgs g{};
        g.A = A[i]; g.B = A[i]; g.ld = kdim[i]; g.M = M[i]; g.N = M[i]; g.kdim = kdim[i]; g.ksplit = ksplit[i];
        g.ntm = g.ntn = (int)((M[i] + T - 1) / T);
        g.lower = 1;
        g.nsplit = nsplit[i];
        g.partial = partial[i];
        const int64_t nwg = (int64_t)g.ntm * (g.ntm + 1) / 2 * nsplit[i];
        if (nwg <= 0) continue;
        if (grp.n == kSyrkGroupMax || total + nwg > (int64_t)UINT32_MAX / 2) flush();
        grp.blk_start[grp.n] = (uint32_t)total;
        grp.g[grp.n++] = g;
        total += nwg;
    }
    flush();
}

// C = A B^T with B lower triangular in (n, k) (B(n, k) = 0 for k > n), both
// row-major over ld = k: the whitening B_fP = sum_{Q <= P} U_fQ Linv_PQ.  M
// rows of A, N rows of B (a multiple of 128), 128-wide tiles, no split.
void launch_gemm_nt_tri(const double *A, const double *B, double *C, int64_t M, int64_t N, int64_t ld,
                        hipStream_t s)
{
    SyrkArgs g{};
    g.A = A; g.B = B; g.ld = ld; g.M = M; g.N = N; g.kdim = ld; g.ksplit = ld;
    g.ntm = (int)((M + 127) / 128);
    g.ntn = (int)((N + 127) / 128);
    g.lower = 0; g.tri_k = 1; g.nsplit = 1;
    g.C = C; g.ldc = ld;
    const int ntiles = g.ntm * g.ntn;
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((k_syrk_f64<128, 4, 2>), dim3((unsigned)ntiles), dim3(512), 0, s, g);
}

}  // namespace dfjk
