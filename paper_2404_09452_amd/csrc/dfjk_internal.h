// Internal declarations of the DF-J/K library: the plan, the device-side
// tables it owns, and the launch wrappers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "dfjk.h"

namespace dfjk {

constexpr int kMaxLAO = 2;     // highest AO angular momentum
constexpr int kMaxLAux = 3;    // highest aux angular momentum
constexpr int kPadAux = 128;   // aux dimension stored as a multiple of this (half-transform tile)
constexpr int kPadF = 64;      // function-pair dimension stored as a multiple of this
constexpr int kMaxPairRows = (2 * kMaxLAO + 1) * (2 * kMaxLAO + 1);   // function pairs of one shell pair

// Int8 slices of the half-transformed tensor (DFJK_MIXED_INT8).  Row mu of X
// is cut into blocks of kI8Block contraction elements; each block has a
// power-of-two scale 2^e (stored as a double) with |x| <= 127/128 2^e, and
// x ~ 2^e sum_{s<kI8Slices} a_s 2^{-7(s+1)}, a_0 in [-127, 127], a_s in
// [-64, 64].  Storage per row: chunks of kI8Chunk elements, each chunk the
// kI8Slices slices one after another ([chunk][slice][64] bytes).  The
// contraction index of a slab runs over column passes of the half transform
// (ht_pass_frags below), then aux rows, then the
// pass's columns (its width rounded up to even, so every pass region is a
// whole number of blocks; the pad column is zero).
constexpr int kTileK = 128;     // K output tile of the split-K partials and the reductions
constexpr int kXcds = 8;        // accelerator complex dies of an MI355X, each with its own L2
constexpr int kI8Slices = 5;
constexpr int kI8Block = 256;
constexpr int kI8Chunk = 64;
constexpr int64_t kI8AutoSlab = 1024;   // largest automatic aux slab of an int8 build

// Half transform: each AO function's partner list (hk_*) is padded to a
// multiple of kHtChunk entries (a padding entry names a real B row and the
// zero coefficient row nao), and the coefficient columns run in passes of at
// most kHtMaxFrag fragments of 16 columns: the fewest passes, the fragments
// spread evenly over them.  The coefficients go to a zero-padded copy of
// nao + 1 rows of ht_ldc(ncol) columns.
constexpr int kHtChunk = 16;
constexpr int kHtMaxFrag = 10;
inline int ht_pass_frags(int64_t ncol)
{
    const int64_t need = (ncol + 15) / 16, passes = (need + kHtMaxFrag - 1) / kHtMaxFrag;
    return passes > 0 ? (int)((need + passes - 1) / passes) : 1;
}
inline int64_t ht_passes(int64_t ncol)
{
    const int64_t f = ht_pass_frags(ncol);
    return ((ncol + 15) / 16 + f - 1) / f;
}
inline int64_t ht_ldc(int64_t ncol) { return ht_passes(ncol) * ht_pass_frags(ncol) * 16; }

// Contraction length of one aux slab of plen rows with ncol columns as the
// precision stores it, and the bytes of its X buffers (main and second plane).
inline bool is_int8(int precision) { return precision == DFJK_MIXED_INT8 || precision == DFJK_MIXED_INT8_FAST; }
inline int64_t x_kdim(int precision, int64_t plen, int64_t ncol)
{
    return plen * (is_int8(precision) ? ncol + (ncol & 1) : ncol);
}
inline size_t x_bytes(int precision, int64_t rows, int64_t kdim)
{
    const size_t n = (size_t)rows * (size_t)kdim;
    switch (precision) {
    case DFJK_FP64: return n * 8;
    case DFJK_MIXED_FP32: return n * 4;
    case DFJK_MIXED_BF16X3: return n * 2;
    default: return n * kI8Slices;
    }
}
inline size_t x_lo_bytes(int precision, int64_t rows, int64_t kdim)
{
    if (precision == DFJK_MIXED_BF16X3) return (size_t)rows * (size_t)kdim * 2;
    if (is_int8(precision)) return (size_t)rows * (size_t)(kdim / kI8Block) * 8;   // block scales
    return 0;
}
inline bool valid_precision(int precision) { return precision >= DFJK_FP64 && precision <= DFJK_MIXED_INT8_FAST; }

// Boys table: F_m(T_k) at T_k = k * h, 0 <= k < kBoysNT, 0 <= m < kBoysNM.
constexpr double kBoysH = 0.05;
constexpr double kBoysTMax = 40.0;
constexpr int kBoysNT = 802;
constexpr int kBoysNM = 24;
constexpr int kBoysMMaxPublic = 16;

// Error carried out of internal routines.
struct Error {
    int code;
    std::string msg;
};

// Shell data as the kernels read it (structure of arrays, device memory).
struct ShellsDev {
    const double *exp;      // exponent
    const double *x, *y, *z;
    const double *norm;     // N_l(exp)
    const double *q;        // Schwarz factor (aux only)
    const int32_t *l;
    const int32_t *off;     // first function
};

// One angular class of significant pairs (la >= lb) or of aux shells.
struct ClassRange {
    int32_t begin, end;
};

// Stages timed by the optional profiler (HIP events on the call's stream).
enum Stage {
    ST_INT3C = 0, ST_METRIC, ST_CHOL, ST_TRTRI, ST_WHITEN,
    ST_DENSITY, ST_J, ST_HALFTRANS, ST_K, ST_KREDUCE,
    ST_BUILD,                           // a whole build on its stream (stages on side streams overlap inside it)
    ST_SETUP,                           // a whole setup on its stream, likewise
    ST_COUNT
};

// One angular class (la >= lb) of the shell pairs of the four-centre direct
// path, as the kernels read it.  Pairs are sorted by descending Schwarz
// factor; entries at and past n are padding.  The Hermite expansion of every
// function pair f = (ma, mb) of pair i is stored twice:
//   Eb[(f * NH + h) * npad + i]         bra layout (pair index fastest)
//   Ek[(i * NF + f) * NH + h]           ket layout, times (-1)^{t+u+v}
// with NF = (2la+1)(2lb+1), NH the Hermite indices (t,u,v) of order <= la+lb.
struct DirectClassDev {
    int32_t n = 0, npad = 0;
    const int32_t *off_a = nullptr, *off_b = nullptr;   // first AO function of each shell
    const int32_t *sh_a = nullptr, *sh_b = nullptr;     // shell indices
    const double *q = nullptr;                          // Schwarz factor
    const double *px = nullptr, *py = nullptr, *pz = nullptr, *p = nullptr;   // product centre, exponent
    const double *Eb = nullptr, *Ek = nullptr;
    int64_t herm_off = 0;   // first double of this class in the per-build Hermite buffers
};

// Host and device state of the four-centre direct path (after dfjk_direct_setup).
struct DirectState {
    bool ready = false;
    std::vector<int32_t> sa[6], sb[6];   // shell pairs per class, orientation la >= lb
    std::vector<double> q[6];
    DirectClassDev cls[6];
    int64_t herm_total = 0;              // doubles of one Hermite buffer (all classes)
    int64_t quartets = 0;                // (bra, ket) pair combinations that pass the screen
    size_t table_bytes = 0;
    char *tables = nullptr;
    const int32_t *fn_shell = nullptr;   // AO function -> shell (device)
    const int32_t *shell_off = nullptr;  // first AO function of each shell, nsh + 1 entries (device)
    const double *boys = nullptr;
    int device = -1;
};

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;       // created on demand, destroyed with the plan
    std::vector<int> rec_stage;         // stage of event pair i (events 2i, 2i+1)
    int open[ST_COUNT];                 // pair of the stage's unfinished begin, or -1
    hipStream_t stream = nullptr;
    Profiler() { for (int &o : open) o = -1; }
    void mark(int stage, bool begin);   // records one event on `stream`
};

struct Plan {
    Profiler prof;
    // ---- molecule (host copies, caller order) ----
    int32_t natm = 0;
    std::vector<double> coords;
    int32_t nsh_ao = 0, nsh_aux = 0;
    std::vector<int32_t> ao_atom, ao_l, ao_off;
    std::vector<double> ao_exp, ao_norm;
    int64_t nao = 0;
    // aux shells in internal order (sorted by l), with the caller index
    std::vector<int32_t> ax_caller;     // internal shell -> caller shell
    std::vector<int32_t> ax_l, ax_off;  // internal order
    std::vector<double> ax_exp, ax_norm, ax_x, ax_y, ax_z;
    std::vector<int32_t> ax_fn_caller;  // internal aux function -> caller aux function
    ClassRange ax_class[kMaxLAux + 1];
    int64_t naux = 0, naux_pad = 0;
    double thresh = 1e-14;
    int32_t aux_slab = 0;               // requested K-build aux slab (0 = automatic)
    int32_t k_tile = 0;                 // requested FP64 K tile (0 = automatic)
    // host-resident B (after dfjk_offload): slab-major pinned copy, the slab
    // width of that layout, and the stream and events of the slab copies
    bool host_B = false;
    const double *hB = nullptr;
    int64_t host_slab = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr}, ev_start = nullptr;
    // second stream of the overlapped half transform and its events
    hipStream_t ht_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_ht[2] = {nullptr, nullptr}, ev_kdone[2] = {nullptr, nullptr};
    hipStream_t j_stream = nullptr;     // side stream: J of a build, the integrals of a setup
    hipEvent_t ev_jfork = nullptr, ev_jdone = nullptr;
    // split counts chosen by dfjk_autotune for the closed-shell C-route build,
    // keyed by nocc * 4 + precision
    std::map<int64_t, int> tuned_nsplit;
    std::map<int64_t, int> tuned_ktile;   // the FP64 K GEMM tile kept with that split count
    int device = 0;
    int num_cus = 256;
    int stage = 0;

    // ---- AO shell table (host, SoA) ----
    std::vector<double> ao_x, ao_y, ao_z;

    // ---- screening results ----
    int64_t npair_all = 0;
    std::vector<double> q_pair;         // every a >= b pair, index a(a+1)/2 + b
    std::vector<double> q_aux;          // internal aux order
    // significant pairs, class sorted; orientation la >= lb
    std::vector<int32_t> sp_a, sp_b, sp_f0;
    std::vector<double> sp_q;
    ClassRange sp_class[6];             // (0,0) (1,0) (1,1) (2,0) (2,1) (2,2)
    int64_t nf = 0, nf_pad = 0, triplets_kept = 0;
    // function-pair rows: AO functions and weight (2 off-diagonal block, 1 diagonal block)
    std::vector<int32_t> f_mu, f_nu;
    std::vector<double> f_w;
    // half-transform lists: for AO function mu, entries hk_off[mu]..hk_off[mu+1]
    std::vector<int32_t> hk_off, hk_row, hk_nu;
    std::vector<int32_t> hk_order;      // AO functions by descending list length

    // ---- four-centre direct path ----
    DirectState dir;

    // ---- resident device workspace (after setup) ----
    char *ws = nullptr;
    size_t ws_bytes = 0;
    struct {
        double *ao_exp, *ao_x, *ao_y, *ao_z, *ao_norm;
        int32_t *ao_l, *ao_off;
        double *ax_exp, *ax_x, *ax_y, *ax_z, *ax_norm, *ax_q;
        int32_t *ax_l, *ax_off, *ax_fn_caller, *ax_fn_internal;
        int32_t *fmap;                  // [nao][nao] -> stored row f, or -1
        int32_t *sp_a, *sp_b, *sp_f0;
        double *sp_q;
        int32_t *f_mu, *f_nu;
        double *f_w;
        int32_t *hk_off, *hk_row, *hk_nu, *hk_order;
        const double *boys;
        double *U, *B, *V, *L, *Linv;
        double *Dinv;                   // inverses of the 64x64 diagonal blocks of L (setup)
        double *pair_rec;               // per shell pair: P, p and the spherical Hermite bra (setup)
        int32_t *status;
    } d{};
};

// ----- layout helpers ------------------------------------------------------
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Carver {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t n) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// ----- host-side tables (generated by the library itself) -------------------
// Real solid harmonics (Racah normalisation) as Cartesian monomial sums:
// coef[l][m][c], Cartesian order lx descending then ly descending.
void solid_harmonic_table(double coef[kMaxLAux + 1][7][10]);
// Boys table F_m(k h) by Gauss-Legendre quadrature of int_0^1 t^{2m} e^{-T t^2} dt.
const std::vector<double> &boys_table();
// Normalisation of a unit-norm solid-harmonic Gaussian.
double shell_norm(int l, double a);

// ----- device constant setup ---------------------------------------------------
// Uploads the solid-harmonic coefficients and the Boys table to the current
// device once; returns the device address of the Boys table.
Error ensure_device_constants(int device, const double **boys_dev);
void upload_boys_table(const double *host, size_t n, const double **dev_addr, hipError_t *err);

// ----- launch wrappers (defined in the .hip files) ---------------------------
// integrals.hip
void launch_boys_eval(int mmax, int64_t n, const double *T, double *F, const double *tab,
                      hipStream_t s);
void launch_schwarz_pairs(int64_t npair, const ShellsDev &ao, const int32_t *dsh, int32_t nd, double *q,
                          hipStream_t s);
void launch_schwarz_aux(int32_t nsh, const ShellsDev &ax, double *q, hipStream_t s);
// Doubles of one shell pair's record for the three-centre kernel: a header of
// 8 (p, P, Schwarz factor) and the bra coefficients [nherm(la+lb)][(2la+1)(2lb+1)],
// rounded up to whole 64-byte lines.
constexpr int pair_rec_doubles(int la, int lb)
{
    return (8 + (la + lb + 1) * (la + lb + 2) * (la + lb + 3) / 6 * (2 * la + 1) * (2 * lb + 1) + 7) / 8 * 8;
}
constexpr int kPairClassLa[6] = {0, 1, 1, 2, 2, 2}, kPairClassLb[6] = {0, 0, 1, 0, 1, 2};
// offset (doubles) of each pair class's records, and the total
void pair_rec_offsets(const Plan &p, int64_t off[7]);
void launch_pair_records(const Plan &p, hipStream_t s);
void launch_pair_records_plans(const Plan *const *plans, int n, hipStream_t s);
void launch_int3c_plans(const Plan *const *plans, int n, hipStream_t s);
void launch_int3c(const Plan &p, hipStream_t s);
bool side_stream(Plan &p);   // jk.hip: p.j_stream with p.ev_jfork / p.ev_jdone
void launch_int3c_rows(const Plan &p, double *U, int64_t f_base, int32_t i0, int32_t i1, hipStream_t s);
void launch_int2c(const Plan &p, hipStream_t s);
void upload_constants(const double coef[kMaxLAux + 1][7][10], hipStream_t s);
// Pair tables of the direct path: for each class, px..p, Eb and Ek from the
// shell lists already in the tables and the AO shell arrays.
void launch_direct_pairs(const DirectClassDev *cls, const ShellsDev &ao, hipStream_t s);

// linalg.hip
void launch_metric_pad(double *V, int64_t n, int64_t npad, hipStream_t s);
void launch_cholesky(double *A, int64_t npad, int32_t *status, double *Dinv, hipStream_t s);
void cholesky_step(double *A, int64_t npad, int64_t k, int32_t *status, double *Dinv, hipStream_t s);
void launch_trtri(double *L, double *Linv, const double *Dinv, int64_t npad, hipStream_t s);
void trtri_begin(double *X, int64_t npad, hipStream_t s);
void trtri_step(const double *L, double *X, const double *Dinv, int64_t npad, int64_t i, hipStream_t s);
void launch_zero_upper(double *L, int64_t npad, hipStream_t s);
void launch_whiten(const double *U, const double *Linv, double *B, int64_t nf_pad, int64_t npad,
                   hipStream_t s);

// jk.hip
struct BuildLayout {
    int64_t nao, naux_pad, nf, ncol;    // ncol = nocc (C route) or nao (D route)
    int precision;
    bool with_D;
    bool delta;                         // K = K0 + X_U X_W^T + (X_U X_W^T)^T
    bool uks;                           // open shell: K_a, K_b from C_a, C_b (ncol = max nocc)
    int32_t nocc_a, nocc_b;
    const double *C0, *K0;              // reference orbitals and K for the increment
    int nsplit_c;
    int ntile;                          // syrk output tiles per side (128 wide)
    int nsplit_k;                       // k splits per slab
    int ktile;                          // FP64 K GEMM tile (128, or 64 written into the 128-wide partials)
    int64_t slab, nslab;                // aux functions per slab (multiple of 128), slab count
    int64_t kdim;                       // slab * ncol: contraction length of one slab
    size_t bytes;
    // offsets into the scratch
    size_t o_D, o_d, o_cpart, o_c, o_X, o_Xlo, o_Bfull, o_X2, o_X2lo, o_U, o_W, o_Kpart, o_Epart, o_Da, o_Db;
    size_t o_Cr, o_align;               // increment: C rotated onto C0, and the alignment's work
    size_t o_Cp, o_Cp2;                 // zero-padded coefficients read by the half transform (two for the increment)
    bool norms;                         // int8: add each slab's digit sums into o_norms (dfjk_build_checked)
    size_t o_norms;
    size_t o_stage[2];                  // staging of host-resident B slabs
    bool overlap;                       // half transform of the next slab beside the K GEMM
    bool j_side;                        // J on a side stream beside the half transform and K
    size_t o_Xb, o_Xblo;                // the second X buffer of the overlapped schedule
};
// nsplit: 0 = the autotuned count when there is one, else the built-in
// choice; -1 = the built-in choice; > 0 = that count (capped by the length)
// force_slab > 0: that many aux functions per slab (a multiple of kPadAux);
// ktile: 0 = the autotuned FP64 K tile when there is one (with nsplit 0),
// else 128; 64 or 128 = that tile
BuildLayout build_layout(const Plan &p, int32_t nocc, int32_t precision, bool with_D, bool delta = false,
                         int nsplit = 0, bool allow_overlap = true, int64_t force_slab = 0, int ktile = 0);
int batch_nsplit(const Plan *const *plans, int n);
void launch_build_batch(int n, Plan *const *plans, const BuildLayout *Ls, const double *const *C, double *const *J,
                        double *const *K, double *const *E, char *const *scratch, hipStream_t s);
BuildLayout build_layout_uks(const Plan &p, int32_t nocc_a, int32_t nocc_b, int32_t precision);
void launch_build(Plan &p, const BuildLayout &L, const double *C, const double *D,
                  double *J, double *K, double *E, char *scratch, hipStream_t s);
void launch_build_uks(Plan &p, const BuildLayout &L, const double *Ca, const double *Cb, double *J, double *Ka,
                      double *Kb, double *E, char *scratch, hipStream_t s);
void launch_build_hostB(Plan &p, const BuildLayout &L, const double *C, double *J, double *K, double *E,
                        char *scratch, hipStream_t s);

// direct.hip: four-centre direct J/K.  Scratch: the density (C route), the
// Hermite density and Hermite J buffers, and the energy partials.
// An incremental build (delta) integrates dD = D - D0 with the
// density-weighted screen and adds the reference J0, K0.
struct DirectLayout {
    bool with_D, delta;
    size_t o_D, o_dsh, o_Dh, o_Jh, o_Epart, bytes;
};
DirectLayout direct_layout(const Plan &p, bool with_D, bool delta = false);
void launch_direct_build(const Plan &p, const DirectLayout &L, const double *C, int32_t nocc, const double *D,
                         const double *D0, const double *J0, const double *K0, double *J, double *K, double *E,
                         char *scratch, hipStream_t s);
void launch_density(const double *C, int64_t nao, int32_t nocc, double scale, double *D, hipStream_t s);

// align.hip: Cr = C Q, Q the orthogonal polar factor of C^T C0 (Procrustes)
// FP64 K contraction by LDS DMA (syrk_f64.hip): split-K partial tiles of
// A B^T, lower tiles or every tile, T = 64 or 128
void launch_syrk_f64(bool lower, const double *A, const double *B, int64_t M, int64_t kdim, int64_t ksplit,
                     int nsplit, int T, double *partial, hipStream_t s);
void launch_syrk_f64_group(int T, int n, const double *const *A, const int64_t *M, const int64_t *kdim,
                           const int64_t *ksplit, const int *nsplit, double *const *partial, hipStream_t s);
void launch_gemm_nt_tri(const double *A, const double *B, double *C, int64_t M, int64_t N, int64_t ld,
                        hipStream_t s);
// Gram bound (align.hip): out[0] = |C^T C|_F, out[1] >= lambda_max(C^T C)
// from |(C^T C)^16|_F^(1/16); work of gram_work_doubles(nocc) doubles.
constexpr int kGramSquarings = 4;
size_t gram_work_doubles(int32_t nocc);
void launch_gram_bound(const double *C, int64_t nao, int32_t nocc, double *work, double *out, hipStream_t s);
// Int8 energy-error bound (bound.hip)
size_t i8_bound_work_doubles(int64_t nao, int32_t nocc);
void launch_i8_norms(const void *X, const double *scales, int64_t nao, int64_t kdim, double *acc, hipStream_t s);
void launch_i8_bound(const double *C, int64_t nao, int32_t nocc, const double *acc, const double *E, int nsums,
                     double *work, double *out, hipStream_t s);
size_t align_work_doubles(int32_t nocc);
void launch_align(const double *C, const double *C0, int64_t nao, int32_t nocc, double *work, double *Cr,
                  hipStream_t s);

// export.hip
void launch_zero(double *p, int64_t n, hipStream_t s);
void launch_zero_rect(double *p, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t c1, hipStream_t s);
void launch_fmap(const Plan &p, hipStream_t s);   // the sampling diagnostic's pair map, from the stored rows
void launch_export(const Plan &p, int kind, double *out, hipStream_t s);
void launch_sample(const Plan &p, int kind, int64_t n, const int32_t *idx, double *out,
                   hipStream_t s);

}  // namespace dfjk
