// Mixed-precision K = X X^T on gfx950 matrix cores (lower output tiles,
// split-K into FP64 partial tiles like the FP64 path).
//
//  FP32:    X stored FP32, v_mfma_f32_16x16x4f32.
//  BF16x3:  X = hi + lo with hi, lo BF16 (hi = rn(x), lo = rn(x - hi));
//           X X^T ~ hi hi^T + hi lo^T + lo hi^T on v_mfma_f32_16x16x32_bf16
//           (the lo lo^T term, ~2^-16 relative, is dropped).
// In both, products accumulate in FP32 over at most kChunk k values and are
// then added into FP64 accumulators, so the FP32 rounding error does not
// grow with the full contraction length (naux * nocc).
//
// f32 MFMA operand layouts (checked on the device):
//   16x16x4 f32:  lane l supplies A[l%16][l/16], B[l/16][l%16];
//   16x16x32 bf16: lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
//                  B[8(l/16) .. +7][l%16];
//   both: accumulator r of lane l is D[4(l/16) + r][l%16].
#include "dfjk_internal.h"

namespace dfjk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4m __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int T = 128;          // output tile
constexpr int kChunk = 512;     // k values per FP32 accumulation chunk

__device__ __forceinline__ void lower_tile(int t, int &tm, int &tn)
{
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    tm = r;
    tn = t - r * (r + 1) / 2;
}

struct SyrkArgs {
    const void *X, *Xlo;
    int64_t ld;        // = kdim
    int64_t M;         // nao
    int64_t kdim, ksplit;
    int ntm;
    double *partial;
};

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_syrk_f32(SyrkArgs g)
{
    constexpr int KC = 32, LDK = KC + 4;
    __shared__ float As[T * LDK], Bs[T * LDK];
    int tm, tn;
    lower_tile(blockIdx.x, tm, tn);
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    const float *X = static_cast<const float *>(g.X);
    const int64_t kb = (int64_t)blockIdx.y * g.ksplit;
    const int64_t ke = min(kb + g.ksplit, g.kdim);

    f64x4m acc[4][4];
    f32x4 a32[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f64x4m{0.0, 0.0, 0.0, 0.0};
            a32[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    int since = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
        for (int it = 0; it < 4; ++it) {           // 128 rows x 32 k = 1024 float4 per operand
            const int idx = tid + 256 * it, row = idx >> 3, kq = (idx & 7) * 4;
            const int64_t m = m0 + row, n = n0 + row;
            float4 va = (m < g.M) ? *reinterpret_cast<const float4 *>(X + m * g.ld + k0 + kq) : float4{0, 0, 0, 0};
            float4 vb = (n < g.M) ? *reinterpret_cast<const float4 *>(X + n * g.ld + k0 + kq) : float4{0, 0, 0, 0};
            *reinterpret_cast<float4 *>(&As[row * LDK + kq]) = va;
            *reinterpret_cast<float4 *>(&Bs[row * LDK + kq]) = vb;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[(wm * 64 + i * 16 + (lane & 15)) * LDK + ks * 4 + (lane >> 4)];
                b[i] = Bs[(wn * 64 + i * 16 + (lane & 15)) * LDK + ks * 4 + (lane >> 4)];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], a32[i][j], 0, 0, 0);
        }
        __syncthreads();
        since += KC;
        if (since >= kChunk || k0 + KC >= ke) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)a32[i][j][r];
                    a32[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            since = 0;
        }
    }
    const int ntiles = g.ntm * (g.ntm + 1) / 2;
    double *dst = g.partial + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (int64_t)(T * T);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm * 64 + i * 16 + 4 * (lane >> 4) + r;
                const int col = wn * 64 + j * 16 + (lane & 15);
                dst[row * T + col] = acc[i][j][r];
            }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_syrk_bf16x3(SyrkArgs g)
{
    constexpr int KC = 32, LDK = KC + 8;   // bf16 elements; row stride 80 bytes
    __shared__ __attribute__((aligned(16))) unsigned short Ah[T * LDK], Al[T * LDK], Bh[T * LDK], Bl[T * LDK];
    int tm, tn;
    lower_tile(blockIdx.x, tm, tn);
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    const unsigned short *Xh = static_cast<const unsigned short *>(g.X);
    const unsigned short *Xl = static_cast<const unsigned short *>(g.Xlo);
    const int64_t kb = (int64_t)blockIdx.y * g.ksplit;
    const int64_t ke = min(kb + g.ksplit, g.kdim);

    f64x4m acc[4][4];
    f32x4 a32[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f64x4m{0.0, 0.0, 0.0, 0.0};
            a32[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    int since = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
        for (int it = 0; it < 2; ++it) {           // 128 rows x 32 k = 512 x 16 bytes per plane
            const int idx = tid + 256 * it, row = idx >> 2, kq = (idx & 3) * 8;
            const int64_t m = m0 + row, n = n0 + row;
            const uint4 z{0, 0, 0, 0};
            uint4 ah = (m < g.M) ? *reinterpret_cast<const uint4 *>(Xh + m * g.ld + k0 + kq) : z;
            uint4 al = (m < g.M) ? *reinterpret_cast<const uint4 *>(Xl + m * g.ld + k0 + kq) : z;
            uint4 bh = (n < g.M) ? *reinterpret_cast<const uint4 *>(Xh + n * g.ld + k0 + kq) : z;
            uint4 bl = (n < g.M) ? *reinterpret_cast<const uint4 *>(Xl + n * g.ld + k0 + kq) : z;
            *reinterpret_cast<uint4 *>(&Ah[row * LDK + kq]) = ah;
            *reinterpret_cast<uint4 *>(&Al[row * LDK + kq]) = al;
            *reinterpret_cast<uint4 *>(&Bh[row * LDK + kq]) = bh;
            *reinterpret_cast<uint4 *>(&Bl[row * LDK + kq]) = bl;
        }
        __syncthreads();
        bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ra = (wm * 64 + i * 16 + (lane & 15)) * LDK + 8 * (lane >> 4);
            const int rb = (wn * 64 + i * 16 + (lane & 15)) * LDK + 8 * (lane >> 4);
            ah[i] = *reinterpret_cast<const bf16x8 *>(&Ah[ra]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&Al[ra]);
            bh[i] = *reinterpret_cast<const bf16x8 *>(&Bh[rb]);
            bl[i] = *reinterpret_cast<const bf16x8 *>(&Bl[rb]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], a32[i][j], 0, 0, 0);
                a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], a32[i][j], 0, 0, 0);
                a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], a32[i][j], 0, 0, 0);
            }
        __syncthreads();
        since += KC;
        if (since >= kChunk || k0 + KC >= ke) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)a32[i][j][r];
                    a32[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            since = 0;
        }
    }
    const int ntiles = g.ntm * (g.ntm + 1) / 2;
    double *dst = g.partial + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (int64_t)(T * T);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm * 64 + i * 16 + 4 * (lane >> 4) + r;
                const int col = wn * 64 + j * 16 + (lane & 15);
                dst[row * T + col] = acc[i][j][r];
            }
}

void launch_syrk_mixed(const BuildLayout &L, const void *X, const void *Xlo, double *part, hipStream_t s)
{
    SyrkArgs g{};
    g.X = X; g.Xlo = Xlo;
    g.ld = L.kdim; g.M = L.nao; g.kdim = L.kdim;
    g.ksplit = (int64_t)align_up((size_t)((L.kdim + L.nsplit_k - 1) / L.nsplit_k), 32);
    g.ntm = L.ntile;
    g.partial = part;
    const int ntiles = L.ntile * (L.ntile + 1) / 2;
    if (L.precision == DFJK_MIXED_FP32)
        hipLaunchKernelGGL(k_syrk_f32, dim3(ntiles, L.nsplit_k), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(k_syrk_bf16x3, dim3(ntiles, L.nsplit_k), dim3(256), 0, s, g);
}

}  // namespace dfjk
