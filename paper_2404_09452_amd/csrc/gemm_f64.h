// FP64 matrix-core tile GEMM for gfx950 (v_mfma_f64_16x16x4f64).
//
//   C[m][n] = alpha * sum_k A[m][k] * Bop(k, n) + beta * C[m][n]
//
// A is row-major with k contiguous.  Bop(k, n) is Bm[n][k] (k contiguous,
// "NT") or Bm[k][n] (n contiguous, "NN").  A TxT output tile is owned by a
// workgroup of WGM x WGN waves; each wave holds (T/WGM) x (T/WGN) of
// accumulators as 16x16 MFMA blocks.  The k loop walks chunks of 16 staged
// through double-buffered LDS (register prefetch of the next chunk, one
// barrier per chunk); inside a chunk the MFMA fragments of the next k step
// are read from LDS before the MFMAs of the current one are issued.
//
// MFMA f64 16x16x4 operand layout on gfx950 (checked on the device):
//   lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   accumulator register r of lane l is D[l/16 + 4r][l%16].
//
// Tiles are enumerated rectangular (tile t -> (t % ntm, t / ntm)) or lower
// triangular (tn <= tm).  Split-K: blockIdx.y selects a k range; with a
// partial buffer the raw TxT tile goes to partial[(split*ntiles + t)*T*T]
// for a fixed-order reduction elsewhere.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dfjk {

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    double *C;
    int64_t ldc;
    int64_t M, N;
    int64_t k_begin, k_end;   // (k_end - k_begin) split in nsplit ranges of ksplit (multiples of 16)
    int64_t ksplit;
    double alpha, beta;
    int32_t lower;            // 1: enumerate tiles with tn <= tm only
    int32_t tri_k;            // 1: Bop(k, n) = 0 for k >= n (stop k at the tile's last column)
    int32_t ntm, ntn;
    double *partial;          // split-K destination, or nullptr
};

constexpr int kGemmKC = 16;

__device__ __forceinline__ void tile_coords(const GemmArgs &g, int t, int &tm, int &tn)
{
    if (g.lower) {
        int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (r * (r + 1) / 2 > t) --r;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        tm = r;
        tn = t - r * (r + 1) / 2;
    } else {
        tm = t % g.ntm;
        tn = t / g.ntm;
        // with tri_k a tile's k range grows with tn: issue the longest first
        if (g.tri_k) tn = g.ntn - 1 - tn;
    }
}

// One output tile (tile, split) of the GEMM g, computed by the calling workgroup.
template <int T, int WGM, int WGN, bool NN>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, const int tile, const int split)
{
    constexpr int NT = 64 * WGM * WGN;                 // threads
    constexpr int KC = kGemmKC, LDS_K = KC + 1;        // padded k stride in LDS
    constexpr int WTM = T / WGM, WTN = T / WGN;        // per-wave tile
    constexpr int MB = WTM / 16, NB = WTN / 16;        // 16x16 blocks per wave
    constexpr int LOADS = T * KC / 2 / NT;             // double2 loads per thread per operand
    static_assert(LOADS * NT * 2 == T * KC, "tile/threads mismatch");
    __shared__ double As[2][T * LDS_K];
    __shared__ double Bs[2][T * LDS_K];

    const int ntiles_all = g.lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntn;
    int tm, tn;
    tile_coords(g, tile, tm, tn);
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;

    int64_t kb = g.k_begin + (int64_t)split * g.ksplit;
    int64_t ke = kb + g.ksplit;
    if (ke > g.k_end) ke = g.k_end;
    if (g.tri_k && ke > n0 + T) ke = n0 + T;

    f64x4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    double2 ra[LOADS], rb[LOADS];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int it = 0; it < LOADS; ++it) {
            const int idx = tid + NT * it;
            {   // A: row idx / (KC/2), k pair idx % (KC/2)
                const int row = idx / (KC / 2), kp = (idx % (KC / 2)) * 2;
                const int64_t m = m0 + row;
                ra[it] = (m < g.M) ? *reinterpret_cast<const double2 *>(g.A + m * g.lda + k0 + kp)
                                   : double2{0.0, 0.0};
            }
            if (!NN) {
                const int row = idx / (KC / 2), kp = (idx % (KC / 2)) * 2;
                const int64_t n = n0 + row;
                rb[it] = (n < g.N) ? *reinterpret_cast<const double2 *>(g.B + n * g.ldb + k0 + kp)
                                   : double2{0.0, 0.0};
            } else {   // B stored [k][n]: k row idx / (T/2), n pair (idx % (T/2)) * 2
                const int kr = idx / (T / 2), np = (idx % (T / 2)) * 2;
                const int64_t n = n0 + np;
                const double *src = g.B + (k0 + kr) * g.ldb + n;
                if (n + 1 < g.N) rb[it] = *reinterpret_cast<const double2 *>(src);
                else rb[it] = double2{n < g.N ? src[0] : 0.0, 0.0};
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int it = 0; it < LOADS; ++it) {
            const int idx = tid + NT * it;
            const int row = idx / (KC / 2), kp = (idx % (KC / 2)) * 2;
            As[buf][row * LDS_K + kp] = ra[it].x;
            As[buf][row * LDS_K + kp + 1] = ra[it].y;
            if (!NN) {
                Bs[buf][row * LDS_K + kp] = rb[it].x;
                Bs[buf][row * LDS_K + kp + 1] = rb[it].y;
            } else {
                const int kr = idx / (T / 2), np = (idx % (T / 2)) * 2;
                Bs[buf][np * LDS_K + kr] = rb[it].x;
                Bs[buf][(np + 1) * LDS_K + kr] = rb[it].y;
            }
        }
    };

    if (kb < ke) {
        load(kb);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = kb; k0 < ke; k0 += KC) {
            const bool more = k0 + KC < ke;
            if (more) load(k0 + KC);
            const double *as = As[buf] + (wm * WTM + (lane & 15)) * LDS_K + (lane >> 4);
            const double *bs = Bs[buf] + (wn * WTN + (lane & 15)) * LDS_K + (lane >> 4);
            double a[2][MB], b[2][NB];
#pragma unroll
            for (int i = 0; i < MB; ++i) a[0][i] = as[i * 16 * LDS_K];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[0][j] = bs[j * 16 * LDS_K];
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                const int cur = ks & 1, nxt = cur ^ 1;
                if (ks + 1 < KC / 4) {
#pragma unroll
                    for (int i = 0; i < MB; ++i) a[nxt][i] = as[i * 16 * LDS_K + (ks + 1) * 4];
#pragma unroll
                    for (int j = 0; j < NB; ++j) b[nxt][j] = bs[j * 16 * LDS_K + (ks + 1) * 4];
                }
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
            }
            if (more) {
                store(buf ^ 1);
                __syncthreads();
                buf ^= 1;
            }
        }
    }

    if (g.partial) {
        double *dst = g.partial + ((int64_t)split * ntiles_all + tile) * (int64_t)(T * T);
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
                const int64_t m = m0 + wm * WTM + i * 16 + (lane >> 4) + 4 * r;
                const int64_t n = n0 + wn * WTN + j * 16 + (lane & 15);
                if (m < g.M && n < g.N) {
                    double *c = g.C + m * g.ldc + n;
                    const double v = g.alpha * acc[i][j][r];
                    *c = (g.beta == 0.0) ? v : v + g.beta * *c;
                }
            }
}

// waves_per_eu 4: at most 128 VGPRs, so two 8-wave workgroups share a CU.
template <int T, int WGM, int WGN, bool NN>
__global__ __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(4)))
void k_gemm_f64(GemmArgs g)
{
    gemm_tile<T, WGM, WGN, NN>(g, blockIdx.x, blockIdx.y);
}

// T = 128 uses eight waves (4 x 2, 32x64 per wave) to keep four waves per
// SIMD resident; T = 64 uses four waves (2 x 2).
template <int T, bool NN>
inline void gemm_f64(GemmArgs g, int nsplit, hipStream_t s)
{
    g.ntm = (int)((g.M + T - 1) / T);
    g.ntn = (int)((g.N + T - 1) / T);
    const int ntiles = g.lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntn;
    if (ntiles <= 0 || nsplit <= 0) return;
    if (T == 128)
        hipLaunchKernelGGL((k_gemm_f64<128, 4, 2, NN>), dim3(ntiles, nsplit), dim3(512), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_f64<64, 2, 2, NN>), dim3(ntiles, nsplit), dim3(256), 0, s, g);
}

}  // namespace dfjk
