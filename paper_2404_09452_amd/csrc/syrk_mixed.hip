// Mixed-precision products for K on gfx950 matrix cores:
//   syrk mode:    P = A A^T on the lower 128x128 tiles      (direct mixed K)
//   general mode: P = A B^T on every 128x128 tile          (incremental K)
// with split-K into FP64 partial tiles summed elsewhere in a fixed order.
//
//  FP32:    operands stored FP32, v_mfma_f32_16x16x4f32.
//  BF16x3:  every operand x stored as hi + lo, both BF16 (hi = rn(x),
//           lo = rn(x - hi)); a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b on
//           v_mfma_f32_16x16x32_bf16 (the lo lo term, ~2^-16 relative, is
//           dropped).
// Products accumulate in FP32 over at most kChunk k values and are then
// added into FP64 accumulators, so FP32 rounding does not grow with the full
// contraction length.  The k loop is pipelined like the FP64 tile GEMM: the
// next chunk is prefetched into registers while the current one is consumed
// from double-buffered LDS, one barrier per chunk.
//
// f32-accumulating MFMA layouts (checked on the device):
//   16x16x4 f32:   lane l supplies A[l%16][l/16], B[l/16][l%16];
//   16x16x32 bf16: lane l supplies A[l%16][8(l/16)..+7], B[8(l/16)..+7][l%16];
//   both: accumulator r of lane l is D[4(l/16) + r][l%16].
#include "dfjk_internal.h"

#include <algorithm>
#include <vector>

namespace dfjk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4m __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int T = 128;          // output tile (four waves, 64x64 each)
constexpr int kChunk = 512;     // k values per FP32 accumulation chunk

__device__ __forceinline__ void mixed_tile(int t, bool lower, int ntm, int &tm, int &tn)
{
    if (lower) {
        int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (r * (r + 1) / 2 > t) --r;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        tm = r;
        tn = t - r * (r + 1) / 2;
    } else {
        tm = t % ntm;
        tn = t / ntm;
    }
}

struct MixedArgs {
    const void *A, *Alo, *B, *Blo;   // [M][ld] planes (lo planes for BF16x3 only)
    int64_t ld;                      // = kdim
    int64_t M;                       // rows of A and of B (nao)
    int64_t kdim, ksplit;
    int ntm;
    int lower;                       // 1: syrk mode (B = A, tiles tn <= tm)
    double *partial;                 // [split][tile][T][T]
};

template <int PREC>
struct MixStage;   // operand chunk staging per precision

// FP32: chunk of KC = 32 k; A and B tiles 128 x 32 floats each.
template <>
struct MixStage<DFJK_MIXED_FP32> {
    static constexpr int KC = 32, LDK = KC + 4;
    static constexpr int SMEM = 2 * 2 * T * LDK;     // floats: [buf][A/B][T*LDK]
};
// BF16x3: chunk of KC = 32 k; four planes (A hi/lo, B hi/lo) of 128 x 32 bf16.
template <>
struct MixStage<DFJK_MIXED_BF16X3> {
    static constexpr int KC = 32, LDK = KC + 8;
    static constexpr int SMEM = 2 * 4 * T * LDK;     // bf16: [buf][plane][T*LDK]
};

template <int PREC>
__global__ __launch_bounds__(256) void k_gemm_mixed(MixedArgs g)
{
    constexpr int KC = MixStage<PREC>::KC, LDK = MixStage<PREC>::LDK;
    using Elem = typename std::conditional<PREC == DFJK_MIXED_FP32, float, unsigned short>::type;
    __shared__ __attribute__((aligned(16))) Elem sm[MixStage<PREC>::SMEM];

    int tm, tn;
    mixed_tile(blockIdx.x, g.lower, g.ntm, tm, tn);
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
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

    // Each thread moves 16-byte pieces: row = idx / (KC*esz/16), column piece idx % (...).
    constexpr int PIECES = KC * (int)sizeof(Elem) / 16;    // 16-byte pieces per row
    constexpr int NP = PREC == DFJK_MIXED_FP32 ? 2 : 4;   // planes
    constexpr int LOADS = T * PIECES / 256;                // pieces per thread per plane
    uint4 reg[NP][LOADS];
    const Elem *src[NP];
    src[0] = static_cast<const Elem *>(g.A);
    src[1] = static_cast<const Elem *>(g.lower ? g.A : g.B);
    if (NP == 4) {
        src[2] = static_cast<const Elem *>(g.Alo);
        src[3] = static_cast<const Elem *>(g.lower ? g.Alo : g.Blo);
    }
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int pl = 0; pl < NP; ++pl) {
            const int64_t r0 = (pl == 1 || pl == 3) ? n0 : m0;
#pragma unroll
            for (int it = 0; it < LOADS; ++it) {
                const int idx = tid + 256 * it, row = idx / PIECES, pc = idx % PIECES;
                const int64_t r = r0 + row;
                reg[pl][it] = (r < g.M)
                    ? *reinterpret_cast<const uint4 *>(src[pl] + r * g.ld + k0 + pc * (16 / sizeof(Elem)))
                    : uint4{0, 0, 0, 0};
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int pl = 0; pl < NP; ++pl)
#pragma unroll
            for (int it = 0; it < LOADS; ++it) {
                const int idx = tid + 256 * it, row = idx / PIECES, pc = idx % PIECES;
                *reinterpret_cast<uint4 *>(&sm[((buf * NP + pl) * T + row) * LDK + pc * (16 / sizeof(Elem))]) =
                    reg[pl][it];
            }
    };

    int since = 0;
    if (kb < ke) {
        load(kb);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = kb; k0 < ke; k0 += KC) {
            const bool more = k0 + KC < ke;
            if (more) load(k0 + KC);
            if constexpr (PREC == DFJK_MIXED_FP32) {
                const float *As = reinterpret_cast<const float *>(sm) + ((buf * 2 + 0) * T) * LDK;
                const float *Bs = reinterpret_cast<const float *>(sm) + ((buf * 2 + 1) * T) * LDK;
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
            } else {
                const unsigned short *P0 = reinterpret_cast<const unsigned short *>(sm) + (buf * 4) * T * LDK;
                const unsigned short *Ah = P0, *Bh = P0 + T * LDK, *Al = P0 + 2 * T * LDK, *Bl = P0 + 3 * T * LDK;
#pragma unroll
                for (int ks = 0; ks < KC / 32; ++ks) {
                    bf16x8 ah[4], al[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = (wm * 64 + i * 16 + (lane & 15)) * LDK + ks * 32 + 8 * (lane >> 4);
                        ah[i] = *reinterpret_cast<const bf16x8 *>(&Ah[o]);
                        al[i] = *reinterpret_cast<const bf16x8 *>(&Al[o]);
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int o = (wn * 64 + j * 16 + (lane & 15)) * LDK + ks * 32 + 8 * (lane >> 4);
                        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&Bh[o]);
                        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&Bl[o]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, a32[i][j], 0, 0, 0);
                            a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, a32[i][j], 0, 0, 0);
                            a32[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, a32[i][j], 0, 0, 0);
                        }
                    }
                }
            }
            since += KC;
            if (since >= kChunk || !more) {
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
            if (more) {
                store(buf ^ 1);
                __syncthreads();
                buf ^= 1;
            }
        }
    }
    const int ntiles = g.lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntm;
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
// Int8 slices (DFJK_MIXED_INT8), the Ozaki splitting of floating-point
// products into exact integer ones (Ozaki, Ogita, Oishi & Rump, Numer.
// Algorithms 59, 2012): with x = 2^{e_x} sum_i a_i 2^{-7(i+1)} and y alike,
//   x y ~ 2^{e_x + e_y} sum_{t=0}^{4} 2^{-7(t+2)} sum_{i+j=t} a_i b_j,
// the products of combined order i + j <= 4 (15 of the 25).  Each order t is
// an exact int32 sum on v_mfma_i32_16x16x64_i8 over one scale block (256 k,
// |sum| < 5 * 127 * 127 * 256 < 2^31), then the five orders are combined in
// FP64 and added with the block's scale 2^{e_x + e_y} into FP64
// accumulators.  The only rounding is the truncation of the slices.
//
// DFJK_MIXED_INT8_FAST (FAST below) keeps the orders i + j <= 3 and the one
// order-4 product a_2 b_2 (11 products; slice a_4 is neither loaded nor
// used).  a_2 b_2 stays because on the diagonal it is a square: dropped, it
// would shift every K_mu mu the same way and bias E_K (by 1e-6 Eh already on
// three waters), whereas the other dropped order-4 products carry no sign.
//
// Workgroup: 128 rows x 64 columns of the output (half of a 128 x 128
// partial tile, blockIdx.x = 2 tile + half), four waves of 64 x 32, each
// 4 x 2 fragments of 16 x 16 with five int32 order accumulators (160
// registers) and FP64 accumulators (64).  One wave per SIMD.  Operands move
// straight from global memory into LDS (global_load_lds_dwordx4, no
// registers): one wave instruction brings one MFMA operand fragment, 16 rows
// x 64 k bytes of one slice, to 1 KB of LDS in lane order, so each later
// fragment read is one contiguous 16-byte read per lane.  A chunk of 64 k is
// 8 NS fragments of the 128 rows and 4 NS of the 64 columns for the NS slices
// used (60 KB at NS = 5); two chunk
// buffers, the next chunk in flight while the current one feeds the MFMAs,
// one barrier per chunk.
// 16x16x64 i8 layout: lane l supplies row l%16 and 16 consecutive k bytes of
// k group l/16 for both operands; accumulator r of lane l is D[4(l/16)+r][l%16].
typedef int i32x4 __attribute__((ext_vector_type(4)));

// s_waitcnt immediates (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt
// 6:4, lgkmcnt 11:8; a field at its maximum does not wait).  Issued through
// the builtin so the compiler's own wait insertion knows what has retired.
constexpr int kWaitVm15 = 15 | (7 << 4) | (15 << 8);             // vmcnt(15)
constexpr int kWaitVm0 = 0 | (7 << 4) | (15 << 8);               // vmcnt(0)
constexpr int kWaitLgkm0 = 15 | (7 << 4) | (0 << 8) | (3 << 14);  // lgkmcnt(0)
constexpr int kI8WavesM = 4;   // waves along the 128 rows: 2 (one wave per SIMD) or 4 (two)

struct I8Args {
    const unsigned char *A, *B;   // [M][kdim / 64][5][64] slices
    const double *sA, *sB;        // [M][kdim / 256] block scales
    int64_t kdim, M, ksplit;      // ksplit: a multiple of kI8Block
    int ntm;
    int lower;
    int nsplit;
    double *partial;              // [split][tile][128][128]
};

// WGM x WGN waves, each RB x CB fragments of 16 x 16 (the workgroup tile
// is always 128 x 64).  Fragments of a chunk are spread over the waves,
// NFW per wave, padded with loads into a spare LDS slot so that every wave
// issues the same count (the vmcnt immediate below).
template <int WGM, int WGN, int RB, int CB, bool FAST>
__device__ __forceinline__ void gemm_i8_tile(I8Args g, unsigned blk)
{
    constexpr int NW = WGM * WGN, NT = 64 * NW;
    constexpr int AR = WGM * RB * 16, BR = WGN * CB * 16;                 // rows of the two operands
    static_assert(AR == T && BR == T / 2, "the workgroup tile is half of a 128 x 128 partial tile");
    constexpr int RBA = AR / 16, RBB = BR / 16;
    constexpr int NS = FAST ? kI8Slices - 1 : kI8Slices;                 // slices loaded
    constexpr int FA = RBA * NS, FB = RBB * NS, NF = FA + FB;           // fragments per chunk
    constexpr int NFW = (NF + NW - 1) / NW, NFS = NFW * NW;              // per wave; slots incl. spares
    constexpr int CH = kI8Slices * kI8Chunk;                             // bytes of one row per chunk
    static_assert(NFW <= 15, "vmcnt immediate holds 4 bits here");
    constexpr int kWaitVmNFW = NFW | (7 << 4) | (15 << 8);              // vmcnt(NFW)
    // two chunk buffers as separate arrays: the compiler can then tell a
    // read of one from a DMA into the other (which buffer is known at
    // compile time below) and does not wait for unrelated loads
    __shared__ __attribute__((aligned(1024))) unsigned char sm0[NFS * 1024];
    __shared__ __attribute__((aligned(1024))) unsigned char sm1[NFS * 1024];

    // workgroup -> (split, tile, half).  With a split count that is a multiple
    // of the XCD count, XCD x (workgroups are dispatched round-robin over the
    // XCDs) runs whole splits x, x + 8, ..., so each XCD's L2 holds one k
    // range of X for every tile of a split.
    const int nth = 2 * (g.lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntm);   // tile halves per split
    int split, th;
    if (g.nsplit % kXcds == 0) {
        const int xcd = blk % kXcds, local = blk / kXcds;
        split = xcd + kXcds * (local / nth);
        th = local % nth;
    } else {
        split = blk / nth;
        th = blk % nth;
    }
    const int half = th & 1, tile = th >> 1;
    int tm, tn;
    mixed_tile(tile, g.lower, g.ntm, tm, tn);
    const int64_t m0 = (int64_t)tm * T, n0 = (int64_t)tn * T + 64 * half;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave / WGN, wn = wave % WGN;
    const int64_t kb = (int64_t)split * g.ksplit;
    const int64_t ke = min(kb + g.ksplit, g.kdim);
    const int64_t rowb = g.kdim * kI8Slices;          // bytes per row
    const int64_t nblk = g.kdim / kI8Block;

    // this lane's byte offset for each fragment its wave loads, relative to
    // the first row of the operand's 128-row tile (which is < M); rows past
    // M read row M-1, whose products only reach outputs that are dropped.
    // Spare slots re-read the first A fragment.  The host keeps 128 rows
    // below 4 GiB.
    const int64_t a0 = m0, b0 = (int64_t)tn * T;
    uint32_t loff[NFW];
#pragma unroll
    for (int q = 0; q < NFW; ++q) {
        const int f = wave + NW * q;
        const bool isA = f < FA || f >= NF;
        const int rb = f >= NF ? 0 : isA ? f % RBA : (f - FA) % RBB;
        const int64_t base = isA ? a0 : b0;
        const int64_t r = min((isA ? m0 : n0) + rb * 16 + (lane & 15), g.M - 1);
        loff[q] = (uint32_t)((r - base) * rowb + 16 * (lane >> 4));
    }
    auto load = [&](int64_t k0, unsigned char *dstbuf) {
        const int64_t cb = (k0 / kI8Chunk) * CH;
#pragma unroll
        for (int q = 0; q < NFW; ++q) {
            const int f = wave + NW * q;
            const bool isA = f < FA || f >= NF;
            const int sl = f >= NF ? 0 : isA ? f / RBA : (f - FA) / RBB;
            const unsigned char *base = (isA ? g.A + a0 * rowb : g.B + b0 * rowb) + cb + sl * kI8Chunk;
            __builtin_amdgcn_global_load_lds((const void *)(base + loff[q]),
                                             (__attribute__((address_space(3))) void *)(dstbuf + f * 1024), 16,
                                             0, 0);
        }
    };

    double acc[RB][CB][4];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

    // Block scales of the 128 rows and 64 columns, staged through LDS one
    // block ahead: thread t < 192 loads its row's (column's) scale of the
    // next block into a register at the start of a block and writes it to
    // ssc[next % 2] at the start of the next block, at least three barriers
    // before the fold of that block reads it.
    __shared__ double ssc[2][AR + BR];
    const int64_t srow_t = tid < AR ? m0 + tid : n0 + (tid - AR);
    const double *sbase_t = tid < AR ? g.sA : g.sB;
    const bool sown = tid < AR + BR && srow_t < g.M;
    double snext = 0.0;
    auto scale_fetch = [&](int64_t blk) {
        snext = (sown && blk < nblk) ? sbase_t[srow_t * nblk + blk] : 0.0;
    };

    // One scale block per iteration: four chunks whose five order sums live
    // only inside the iteration (the first chunk starts them from zero), then
    // their FP64 fold.  Chunks run two ahead: a chunk's fragments are read
    // from LDS into registers first, then (after a barrier: every wave has
    // read that buffer) the DMA of the chunk two ahead goes into the same
    // buffer, then the MFMAs run.  The DMA of the next chunk was issued one
    // chunk earlier; waiting for it leaves the NFW newer loads of each wave
    // in flight (vmcnt counts a wave's loads and they retire in order).
    // Barriers without memory fences keep those loads outstanding across them.
    const int64_t nch = (ke - kb) / kI8Chunk;
    if (kb < ke) {
        scale_fetch(kb / kI8Block);
        // every chunk step issues one DMA (past the end: the last chunk again,
        // never read), so each wait below keeps exactly one chunk in flight
        auto chunk_k = [&](int64_t ci) { return kb + min(ci, nch - 1) * kI8Chunk; };
        load(chunk_k(0), sm0);
        load(chunk_k(1), sm1);
        __builtin_amdgcn_s_waitcnt(kWaitVmNFW);
        __builtin_amdgcn_s_barrier();
        for (int64_t k0 = kb; k0 < ke; k0 += kI8Block) {
            const int64_t blk = k0 / kI8Block;
            if (tid < AR + BR) ssc[blk & 1][tid] = snext;
            scale_fetch(blk + 1);
            i32x4 lev[kI8Slices][RB][CB];   // order sums t = 0..4
#pragma unroll
            for (int c = 0; c < kI8Block / kI8Chunk; ++c) {
                const int64_t ci = (k0 - kb) / kI8Chunk + c;     // chunk index in this split (ci % 2 == c % 2)
                unsigned char *cur = (c & 1) ? sm1 : sm0;
                const unsigned char *Fa = cur + (wm * RB) * 1024 + lane * 16;
                const unsigned char *Fb = cur + (FA + wn * CB) * 1024 + lane * 16;
                i32x4 bf[NS][CB], af[NS][RB];
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
#pragma unroll
                    for (int j = 0; j < CB; ++j)
                        bf[sl][j] = *reinterpret_cast<const i32x4 *>(Fb + (sl * RBB + j) * 1024);
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        af[sl][i] = *reinterpret_cast<const i32x4 *>(Fa + (sl * RBA + i) * 1024);
                }
                __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                __builtin_amdgcn_s_barrier();
                load(chunk_k(ci + 2), cur);
                __builtin_amdgcn_sched_barrier(0);   // the DMA goes out before the MFMAs
#pragma unroll
                for (int si = 0; si < NS; ++si)
#pragma unroll
                    for (int sj = 0; sj < NS; ++sj)
#pragma unroll
                        for (int i = 0; i < RB; ++i)
#pragma unroll
                            for (int j = 0; j < CB; ++j) {
                                const bool kept = FAST ? si + sj <= 3 || (si == 2 && sj == 2) : si + sj <= 4;
                                if (!kept) continue;
                                // the first product of each order sum in a block starts it from zero
                                const bool first = c == 0 && si == (FAST && si + sj == 4 ? 2 : 0);
                                const i32x4 cin = first ? i32x4{0, 0, 0, 0} : lev[si + sj][i][j];
                                lev[si + sj][i][j] =
                                    __builtin_amdgcn_mfma_i32_16x16x64_i8(af[si][i], bf[sj][j], cin, 0, 0, 0);
                            }
                __builtin_amdgcn_sched_barrier(0);   // and the wait stays after them
                __builtin_amdgcn_s_waitcnt(kWaitVmNFW);
                __builtin_amdgcn_s_barrier();
            }
            // FP64 fold: sum_t 2^{-7t} (order t sum) times the block scales
            const double *sc = ssc[blk & 1];
            double sb[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) sb[j] = sc[AR + (wn * CB + j) * 16 + (lane & 15)] * 0x1p-14;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                double sa[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) sa[r] = sc[(wm * RB + i) * 16 + 4 * (lane >> 4) + r];
#pragma unroll
                for (int j = 0; j < CB; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double v = (double)lev[4][i][j][r];
#pragma unroll
                        for (int t = 3; t >= 0; --t) v = fma(v, 0x1p-7, (double)lev[t][i][j][r]);
                        acc[i][j][r] = fma(v, sa[r] * sb[j], acc[i][j][r]);
                    }
            }
        }
        __builtin_amdgcn_s_waitcnt(kWaitVm0);   // no DMA into LDS outlives the workgroup
    }
    double *dst = g.partial + ((int64_t)split * (nth / 2) + tile) * (int64_t)(T * T) + 64 * half;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (wm * RB + i) * 16 + 4 * (lane >> 4) + r;
                const int col = (wn * CB + j) * 16 + (lane & 15);
                dst[row * T + col] = acc[i][j][r];
            }
}

template <int WGM, int WGN, int RB, int CB, bool FAST>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(WGM * WGN / 4, WGM * WGN / 4)))
void k_gemm_i8(I8Args g)
{
    gemm_i8_tile<WGM, WGN, RB, CB, FAST>(g, blockIdx.x);
}

// The int8 K of several molecules in one launch (batches): workgroup b runs
// workgroup b - blk_start[m] of molecule m's own launch, descriptors by value.
constexpr int kI8GroupMax = 16;
struct I8Group {
    int32_t n;
    uint32_t blk_start[kI8GroupMax + 1];
    I8Args g[kI8GroupMax];
};
static_assert(sizeof(I8Group) <= 4096, "kernel arguments are limited to 4 KB");

template <int WGM, int WGN, int RB, int CB, bool FAST>
__global__ __launch_bounds__(64 * WGM * WGN)
__attribute__((amdgpu_waves_per_eu(WGM * WGN / 4, WGM * WGN / 4)))
void k_gemm_i8_group(I8Group grp)
{
    int m = 0;
    while (m + 1 < grp.n && blockIdx.x >= grp.blk_start[m + 1]) ++m;
    gemm_i8_tile<WGM, WGN, RB, CB, FAST>(grp.g[m], blockIdx.x - grp.blk_start[m]);
}

// Split count of the int8 K: workgroups run one per CU, all with the same
// k length, so the time is (rounds of workgroups) x (k per split).  Counts
// that are multiples of the XCD count run whole splits per XCD (rounds
// counted per XCD); smaller k lengths fall back to any count.  The smallest
// count within 2% of the best wins; at least 4 scale blocks per split.
int i8_nsplit(int64_t nao, int64_t kdim, bool lower, int num_cus)
{
    const int ntm = (int)((nao + T - 1) / T);
    const int64_t wg = 2 * (int64_t)(lower ? ntm * (ntm + 1) / 2 : ntm * ntm);
    const int slots = num_cus > 0 ? num_cus : 256;
    const int xslots = std::max(1, slots / kXcds);
    const int64_t nblk = kdim / kI8Block;
    const int maxs = (int)std::max<int64_t>(1, std::min<int64_t>(64, nblk / 4));
    std::vector<double> cost(maxs + 1, 1e300);
    double best = 1e300;
    for (int ns = 1; ns <= maxs; ++ns) {
        const int64_t per = (nblk + ns - 1) / ns;
        const int64_t rounds = ns % kXcds == 0 ? (wg * (ns / kXcds) + xslots - 1) / xslots
                                               : (wg * ns + slots - 1) / slots;
        cost[ns] = (double)rounds * (double)per;
        best = std::min(best, cost[ns]);
    }
    // a split count that is a multiple of the XCD count runs whole splits per
    // XCD, so the tiles of one k range share their panels in one L2 while
    // they run together: the cheapest such count is taken when within 15% of
    // the best and a split's workgroups fill at most four rounds of one XCD
    // (32-water cluster, 72 workgroups per split: 7 splits in turn 9.2-9.5 ms
    // per build, 8 / 16 / 32 / 64 whole splits per XCD 9.76 / 9.22 / 8.97 /
    // 9.05 ms; 128-water cluster, 930 per split: 3 splits in turn 1.15 s, 8
    // per XCD 1.21 s)
    int bx = 0;
    if (wg <= 4 * xslots)
        for (int ns = kXcds; ns <= maxs; ns += kXcds)
            if (bx == 0 || cost[ns] < cost[bx]) bx = ns;
    if (bx > 0 && cost[bx] <= 1.15 * best) return bx;
    for (int ns = 1; ns <= maxs; ++ns)
        if (cost[ns] <= 1.02 * best) return ns;
    return 1;
}

void launch_gemm_i8(bool lower, const void *A, const double *sA, const void *B, const double *sB, int64_t nao,
                    int64_t kdim, int nsplit, bool fast, double *part, hipStream_t s)
{
    I8Args g{};
    g.A = static_cast<const unsigned char *>(A);
    g.B = static_cast<const unsigned char *>(B);
    g.sA = sA; g.sB = sB;
    g.kdim = kdim; g.M = nao;
    g.ntm = (int)((nao + T - 1) / T);
    g.lower = lower ? 1 : 0;
    g.ksplit = (int64_t)align_up((size_t)(((kdim / kI8Block) + nsplit - 1) / nsplit), 1) * kI8Block;
    g.partial = part;
    g.nsplit = nsplit;
    const int ntiles = lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntm;
    const dim3 grid(2 * ntiles * nsplit), block(64 * 2 * kI8WavesM);
    if (fast)
        hipLaunchKernelGGL((k_gemm_i8<kI8WavesM, 2, 8 / kI8WavesM, 2, true>), grid, block, 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_i8<kI8WavesM, 2, 8 / kI8WavesM, 2, false>), grid, block, 0, s, g);
}

// Lower-tile int8 K partials of several molecules (one X and its block
// scales each, kdim[i] long, nsplit[i] splits), as launch_gemm_i8 lays them
// out, in launches of up to kI8GroupMax molecules.
void launch_gemm_i8_group(bool fast, int n, const void *const *X, const double *const *sX, const int64_t *nao,
                          const int64_t *kdim, const int *nsplit, double *const *part, hipStream_t s)
{
    I8Group grp{};
    int64_t total = 0;
    const dim3 block(64 * 2 * kI8WavesM);
    auto flush = [&]() {
        if (grp.n == 0) return;
        grp.blk_start[grp.n] = (uint32_t)total;
        if (fast)
            hipLaunchKernelGGL((k_gemm_i8_group<kI8WavesM, 2, 8 / kI8WavesM, 2, true>), dim3((unsigned)total), block,
                               0, s, grp);
        else
            hipLaunchKernelGGL((k_gemm_i8_group<kI8WavesM, 2, 8 / kI8WavesM, 2, false>), dim3((unsigned)total), block,
                               0, s, grp);
        grp = I8Group{};
        total = 0;
    };
    for (int i = 0; i < n; ++i) {
        I8Args g{};
        g.A = static_cast<const unsigned char *>(X[i]);
        g.B = g.A;
        g.sA = sX[i]; g.sB = sX[i];
        g.kdim = kdim[i]; g.M = nao[i];
        g.ntm = (int)((nao[i] + T - 1) / T);
        g.lower = 1;
        g.ksplit = (int64_t)align_up((size_t)(((kdim[i] / kI8Block) + nsplit[i] - 1) / nsplit[i]), 1) * kI8Block;
        g.partial = part[i];
        g.nsplit = nsplit[i];
        const int64_t nwg = 2 * (int64_t)(g.ntm * (g.ntm + 1) / 2) * nsplit[i];
        if (nwg <= 0) continue;
        if (grp.n == kI8GroupMax || total + nwg > (int64_t)UINT32_MAX / 2) flush();
        grp.blk_start[grp.n] = (uint32_t)total;
        grp.g[grp.n++] = g;
        total += nwg;
    }
    flush();
}

// Split count: one round of workgroups (two per CU), each split a multiple
// of the chunk of the precision and at least 512 k long.
static int mixed_splits(int ntiles, int64_t kdim, int num_cus)
{
    const int slots = 2 * (num_cus > 0 ? num_cus : 256);
    int ns = ntiles >= slots ? 1 : slots / ntiles;
    const int64_t maxs = kdim / 512;
    if (ns > maxs) ns = (int)(maxs > 0 ? maxs : 1);
    return ns < 1 ? 1 : ns;
}

int mixed_nsplit(int64_t nao, int64_t kdim, bool lower, int num_cus)
{
    const int ntm = (int)((nao + T - 1) / T);
    return mixed_splits(lower ? ntm * (ntm + 1) / 2 : ntm * ntm, kdim, num_cus);
}

void launch_gemm_mixed(int precision, bool lower, const void *A, const void *Alo, const void *B, const void *Blo,
                       int64_t nao, int64_t kdim, int nsplit, double *part, hipStream_t s)
{
    MixedArgs g{};
    g.A = A; g.Alo = Alo; g.B = B; g.Blo = Blo;
    g.ld = kdim; g.M = nao; g.kdim = kdim;
    g.ntm = (int)((nao + T - 1) / T);
    g.lower = lower ? 1 : 0;
    const int kc = precision == DFJK_MIXED_FP32 ? MixStage<DFJK_MIXED_FP32>::KC : MixStage<DFJK_MIXED_BF16X3>::KC;
    g.ksplit = (int64_t)align_up((size_t)((kdim + nsplit - 1) / nsplit), kc);
    g.partial = part;
    const int ntiles = lower ? g.ntm * (g.ntm + 1) / 2 : g.ntm * g.ntm;
    if (precision == DFJK_MIXED_FP32)
        hipLaunchKernelGGL(k_gemm_mixed<DFJK_MIXED_FP32>, dim3(ntiles, nsplit), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(k_gemm_mixed<DFJK_MIXED_BF16X3>, dim3(ntiles, nsplit), dim3(256), 0, s, g);
}

}  // namespace dfjk
