// Four-centre direct J/K on gfx950: exact (unfitted) Coulomb and exchange
// from Schwarz-screened two-electron integrals over shell quartets, the
// direct-SCF path the package began with (paper, Introduction; "Limitations
// and Future Development: Direct SCF & Other Integral Schemes").  The paper's
// kernels use Rys quadrature; here the integrals are McMurchie-Davidson on
// the Hermite tables the three-centre kernels already use, in the split that
// gives a J-engine for Coulomb:
//
//   (ab|cd) = pref sum_h E^{ab}_f[h] sum_k (-1)^{|k|} E^{cd}_g[k] R_{h+k}(alpha, P - Q),
//   pref = 2 pi^{5/2} / (p q sqrt(p+q)),  alpha = p q / (p+q).
//
// J.  With the ket density in Hermite form, Dh_cd[k] = w (-1)^{|k|} sum_g E^{cd}_g[k] D_g
// (w = 2 for c != d: both orders of the pair), every quartet adds
// pref sum_k R_{h+k} Dh_cd[k] to a Hermite J vector Jh_ab[h] of the bra pair,
// which a thread keeps in registers over its ket loop; J_f = sum_h E^{ab}_f[h] Jh_ab[h].
//
// K.  K_{mu nu} = sum (mu la|nu si) D_{la si}.  A visit of bra pair {a,b}
// and ket pair {c,d} forms the integral block and adds its contractions
// to the blocks K_ac (with D_bd), K_ad (D_bc), K_bc (D_ad) and K_bd (D_ac),
// leaving out the duplicates of a = b or c = d.  Every ordered (bra, ket)
// combination of pairs is visited, so the block K_xy (x in {a,b}, y in
// {c,d}) of shells x > y also arrives, transposed, from the visit with bra
// and ket swapped: only blocks with shell x >= y are written (FP64 atomics)
// and the upper triangle is mirrored at the end.
//
// Mapping.  One wave of 64 lanes per launch block.  Light quartet classes:
// lane = bra pair of one class, pairs sorted by descending Schwarz factor,
// and the ket loop (pairs of one class, also sorted) is the same for every
// lane, so its data are uniform loads.  Heavy classes (la+lb+lc+ld >= 5, or
// la = 2 with few pairs: much work per quartet): a wave takes 8 bra pairs x 8 ket pairs
// per step and blockIdx.z takes one row of the first bra shell.  The ket
// loop stops for the whole wave at the first step whose leading ket pair
// has Q_cd * Q_max(wave) below the threshold; lanes whose own bound fails
// sit out that step.  blockIdx.y splits the ket range into short pieces so
// that a launch has many waves; the Hermite J vectors of the splits are
// summed with FP64 atomics.
#include "dfjk_internal.h"
#include "hermite.h"

namespace dfjk {

DirectLayout direct_layout(const Plan &p, bool with_D, bool delta)
{
    DirectLayout L{};
    L.with_D = with_D;
    L.delta = delta;
    size_t off = 0;
    auto take = [&](size_t b) { off = align_up(off, 256); size_t o = off; off += b; return o; };
    L.o_D = (with_D && !delta) ? 0 : take((size_t)p.nao * p.nao * 8);   // D from C, or D - D0
    L.o_dsh = delta ? take(((size_t)p.nsh_ao * p.nsh_ao + 1) * 8) : 0;   // block maxima, then the overall max
    L.o_Dh = take((size_t)std::max<int64_t>(p.dir.herm_total, 1) * 8);
    L.o_Jh = take((size_t)std::max<int64_t>(p.dir.herm_total, 1) * 8);
    L.o_Epart = take((size_t)2 * 256 * 8);
    L.bytes = align_up(off, 256);
    return L;
}

__global__ void k_dfill(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static void dfill(double *p, int64_t n, hipStream_t s)
{
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
    if (n > 0) hipLaunchKernelGGL(k_dfill, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0, s, p, n, 0.0);
}

// Read of a table entry whose index is the same for every lane of the wave,
// through the constant address space so that it becomes a scalar load (the
// tables are read only for the whole kernel).  Tables written by an earlier
// kernel on the stream are visible: caches are invalidated between kernels.
template <class T>
__device__ __forceinline__ T uniform_load(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)(p);
}

// dD = D - D0, and the largest |dD| over each block of shells (x, y), taken
// over both orientations (the density-weighted Schwarz bound of a quartet).
__global__ void k_dsub(const double *__restrict__ D, const double *__restrict__ D0, int64_t n,
                       double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = D[i] - D0[i];
}

__global__ void k_shell_dmax(const double *__restrict__ dD, int64_t nao, int32_t nsh, const int32_t *__restrict__ off,
                             double *__restrict__ dsh)
{
    const int64_t xy = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (xy >= (int64_t)nsh * nsh) return;
    const int x = (int)(xy / nsh), y = (int)(xy % nsh);
    double m = 0.0;
    for (int mu = off[x]; mu < off[x + 1]; ++mu)
        for (int nu = off[y]; nu < off[y + 1]; ++nu)
            m = fmax(m, fmax(fabs(dD[(int64_t)mu * nao + nu]), fabs(dD[(int64_t)nu * nao + mu])));
    dsh[xy] = m;
}

// dsh[nsh * nsh] = the largest entry of the table (one block, fixed order).
__global__ __launch_bounds__(256) void k_dmax_all(double *__restrict__ dsh, int64_t n)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, dsh[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dsh[n] = red[0];
}

// Hermite density of every pair of one class (ket layout, signed).
template <int LA, int LB>
__global__ __launch_bounds__(128) void k_dherm(DirectClassDev c, const double *__restrict__ D, int64_t nao,
                                               double *__restrict__ Dh)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, LAB = LA + LB, NH = nherm(LAB);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    const int oa = c.off_a[i], ob = c.off_b[i];
    const bool same = c.sh_a[i] == c.sh_b[i];
    double d[NA * NB];
#pragma unroll
    for (int ma = 0; ma < NA; ++ma)
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
            const double v = D[(int64_t)(oa + ma) * nao + ob + mb];
            d[ma * NB + mb] = same ? v : v + D[(int64_t)(ob + mb) * nao + oa + ma];
        }
    double *out = Dh + c.herm_off + (int64_t)i * NH;
#pragma unroll
    for (int t = 0; t <= LAB; ++t)
#pragma unroll
        for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= LAB; ++v) {
                const int h = hidx(t, u, v);
                double s = 0.0;
#pragma unroll
                for (int f = 0; f < NA * NB; ++f) s += c.Eb[(int64_t)(f * NH + h) * c.npad + i] * d[f];
                out[h] = ((t + u + v) & 1) ? -s : s;
            }
}

// Shape of the work of one quartet class: the plain shape gives each lane
// its own bra pair against a ket pair that is the same for the whole wave;
// the tiled shape (for heavy classes: few pairs, much work per quartet) gives
// a wave an 8 x 8 tile of (bra, ket) pairs, so that a handful of pairs still
// fills the lanes, and splits the rows of the first bra shell over blockIdx.z.
template <bool TILED, int LA>
struct QuartetShape {
    static constexpr int NA = 2 * LA + 1;
    static constexpr bool heavy = TILED;
    static constexpr int TK = heavy ? 8 : 1;       // ket pairs per wave iteration
    static constexpr int TB = 64 / TK;             // bra pairs per wave
    static constexpr bool split_a = heavy && NA > 1;
};

// The integral kernel for bra class (LA, LB) and ket class (LC, LD).
template <int LA, int LB, int LC, int LD, bool TILED>
__global__ __launch_bounds__(64) void k_direct(DirectClassDev bra, DirectClassDev ket, int32_t kchunk, double tau,
                                               const double *__restrict__ boys_tab, const double *__restrict__ D,
                                               int64_t nao, const double *__restrict__ Dh, double *__restrict__ Jh,
                                               double *__restrict__ K, int32_t with_k,
                                               const double *__restrict__ dsh, int32_t nsh)
{
    constexpr int LAB = LA + LB, LCD = LC + LD, L = LAB + LCD;
    constexpr int NHB = nherm(LAB), NHK = nherm(LCD);
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NC = 2 * LC + 1, ND = 2 * LD + 1;
    constexpr int NFB = NA * NB, NFK = NC * ND;
    using S = QuartetShape<TILED, LA>;
    constexpr int TK = S::TK, TB = S::TB;
    // Small bra classes: the rows of a unrolled and the bra Hermite table kept
    // in registers over the ket loop; larger ones loop over the rows of a at
    // run time (or take one row per blockIdx.z) and read the table per use.
    constexpr int kUnrollA = NFB <= 3 ? NA : 1;
    constexpr bool kHoist = NFB <= 3 && !S::split_a;

    const int lane = threadIdx.x, ib = lane / TK, jk = lane % TK;
    const int i = blockIdx.x * TB + ib;
    const bool valid = i < bra.n;
    const int j0 = blockIdx.y * kchunk;
    const int j1 = min(ket.n, j0 + kchunk);
    if (j0 >= j1) return;
    // the Schwarz bound of the loop ends: Q_ab Q_cd, times the largest
    // |D - D0| anywhere for an incremental build
    const double qwave = uniform_load(bra.q + blockIdx.x * TB) *
                         (dsh ? uniform_load(dsh + (int64_t)nsh * nsh) : 1.0);   // largest bound of this wave
    if (!(uniform_load(ket.q + j0) * qwave >= tau)) return;
    const int ma0 = S::split_a ? (int)blockIdx.z : 0;
    const int ma1 = S::split_a ? ma0 + 1 : NA;
    const bool do_j = !S::split_a || blockIdx.z == 0;

    const int ic = valid ? i : blockIdx.x * TB;
    const double qa = bra.q[ic];
    const double p = bra.p[ic], Px = bra.px[ic], Py = bra.py[ic], Pz = bra.pz[ic];
    const int oa = bra.off_a[ic], ob = bra.off_b[ic], sa = bra.sh_a[ic], sb = bra.sh_b[ic];
    const bool ab_same = sa == sb;

    double ebr[kHoist ? NFB * NHB : 1];
    if constexpr (kHoist) {
#pragma unroll
        for (int x = 0; x < NFB * NHB; ++x) ebr[x] = bra.Eb[(int64_t)x * bra.npad + ic];
    }
    double jh[NHB];
#pragma unroll
    for (int h = 0; h < NHB; ++h) jh[h] = 0.0;
    bool any = false;

    // ket entries: scalar loads when the whole wave reads the same pair
    auto kd = [&](const double *t, int64_t x) -> double {
        if constexpr (TK == 1) return uniform_load(t + x);
        else return t[x];
    };
    auto ki = [&](const int32_t *t, int64_t x) -> int32_t {
        if constexpr (TK == 1) return uniform_load(t + x);
        else return t[x];
    };
    for (int jt = j0; jt < j1; jt += TK) {
        if (!(uniform_load(ket.q + jt) * qwave >= tau)) break;   // the first ket of a step is its largest
        const int j = jt + jk;
        if (!(valid && j < j1 && qa * kd(ket.q, j) >= tau)) continue;
        if (dsh) {
            // density-weighted bound: Q_ab Q_cd times the largest |dD| of the
            // blocks this quartet contracts with (cd for J; bd, bc, ad, ac for K)
            const int64_t jc = ki(ket.sh_a, j), jd = ki(ket.sh_b, j);
            const double dm = fmax(fmax(dsh[jc * nsh + jd], fmax(dsh[(int64_t)sb * nsh + jd], dsh[(int64_t)sb * nsh + jc])),
                                   fmax(dsh[(int64_t)sa * nsh + jd], dsh[(int64_t)sa * nsh + jc]));
            if (!(qa * kd(ket.q, j) * dm >= tau)) continue;
        }
        any = true;
        const double q = kd(ket.p, j);
        const double X = Px - kd(ket.px, j), Y = Py - kd(ket.py, j), Z = Pz - kd(ket.pz, j);
        const double pq = p + q, alpha = p * q / pq;
        double F[L + 1];
        boys<L>(alpha * (X * X + Y * Y + Z * Z), F, boys_tab);
        double R[nherm(L)];
        hermite_R<L>(alpha, X, Y, Z, F, R);
        const double pref = kTwoPi52 / (p * q * sqrt(pq));

        // Coulomb: Jh[h] += pref sum_k R[h + k] Dh[k]
        if (do_j) {
            const double *dh = Dh + ket.herm_off + (int64_t)j * NHK;
#pragma unroll
            for (int t = 0; t <= LAB; ++t)
#pragma unroll
                for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
                    for (int v = 0; v + u + t <= LAB; ++v) {
                        double s = 0.0;
#pragma unroll
                        for (int t2 = 0; t2 <= LCD; ++t2)
#pragma unroll
                            for (int u2 = 0; u2 + t2 <= LCD; ++u2)
#pragma unroll
                                for (int v2 = 0; v2 + u2 + t2 <= LCD; ++v2)
                                    s += R[hidx(t + t2, u + u2, v + v2)] * kd(dh, hidx(t2, u2, v2));
                        jh[hidx(t, u, v)] += pref * s;
                    }
        }
        if (!with_k) continue;

        // Exchange
        const int oc = ki(ket.off_a, j), od = ki(ket.off_b, j), sc = ki(ket.sh_a, j), sd = ki(ket.sh_b, j);
        const bool cd_same = sc == sd;
        const bool w_ac = sa >= sc, w_ad = !cd_same && sa >= sd;
        const bool w_bc = !ab_same && sb >= sc, w_bd = !ab_same && !cd_same && sb >= sd;
        if (!(w_ac || w_ad || w_bc || w_bd)) continue;
        const double *ek = ket.Ek + (int64_t)j * NFK * NHK;
        // rows of b: over every ma of this thread in registers (one row of a
        // per thread: flushed per mb instead)
        double kbc[S::split_a ? 1 : NB][NC], kbd[S::split_a ? 1 : NB][ND];
        if constexpr (!S::split_a) {
#pragma unroll
            for (int x = 0; x < NB; ++x) {
#pragma unroll
                for (int y = 0; y < NC; ++y) kbc[x][y] = 0.0;
#pragma unroll
                for (int y = 0; y < ND; ++y) kbd[x][y] = 0.0;
            }
        }
#pragma unroll kUnrollA
        for (int ma = ma0; ma < ma1; ++ma) {
            double kac[NC], kad[ND];
#pragma unroll
            for (int y = 0; y < NC; ++y) kac[y] = 0.0;
#pragma unroll
            for (int y = 0; y < ND; ++y) kad[y] = 0.0;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) {
                const int f = ma * NB + mb;
                // V[k] = sum_h E_f[h] R[h + k]
                double V[NHK];
#pragma unroll
                for (int k = 0; k < NHK; ++k) V[k] = 0.0;
#pragma unroll
                for (int t = 0; t <= LAB; ++t)
#pragma unroll
                    for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
                        for (int v = 0; v + u + t <= LAB; ++v) {
                            const int h = hidx(t, u, v);
                            double e;
                            if constexpr (kHoist) e = ebr[f * NHB + h];
                            else e = bra.Eb[(int64_t)(f * NHB + h) * bra.npad + ic];
#pragma unroll
                            for (int t2 = 0; t2 <= LCD; ++t2)
#pragma unroll
                                for (int u2 = 0; u2 + t2 <= LCD; ++u2)
#pragma unroll
                                    for (int v2 = 0; v2 + u2 + t2 <= LCD; ++v2)
                                        V[hidx(t2, u2, v2)] += e * R[hidx(t + t2, u + u2, v + v2)];
                        }
                double rbc[NC], rbd[ND];
#pragma unroll
                for (int y = 0; y < NC; ++y) rbc[y] = 0.0;
#pragma unroll
                for (int y = 0; y < ND; ++y) rbd[y] = 0.0;
#pragma unroll
                for (int mc = 0; mc < NC; ++mc)
#pragma unroll
                    for (int md = 0; md < ND; ++md) {
                        const int g = mc * ND + md;
                        double I = 0.0;
#pragma unroll
                        for (int k = 0; k < NHK; ++k) I += kd(ek, g * NHK + k) * V[k];
                        I *= pref;
                        kac[mc] += I * D[(int64_t)(ob + mb) * nao + od + md];
                        kad[md] += I * D[(int64_t)(ob + mb) * nao + oc + mc];
                        rbc[mc] += I * D[(int64_t)(oa + ma) * nao + od + md];
                        rbd[md] += I * D[(int64_t)(oa + ma) * nao + oc + mc];
                    }
                if constexpr (S::split_a) {
                    if (w_bc)
#pragma unroll
                        for (int y = 0; y < NC; ++y) unsafeAtomicAdd(&K[(int64_t)(ob + mb) * nao + oc + y], rbc[y]);
                    if (w_bd)
#pragma unroll
                        for (int y = 0; y < ND; ++y) unsafeAtomicAdd(&K[(int64_t)(ob + mb) * nao + od + y], rbd[y]);
                } else {
#pragma unroll
                    for (int y = 0; y < NC; ++y) kbc[mb][y] += rbc[y];
#pragma unroll
                    for (int y = 0; y < ND; ++y) kbd[mb][y] += rbd[y];
                }
            }
            if (w_ac)
#pragma unroll
                for (int y = 0; y < NC; ++y) unsafeAtomicAdd(&K[(int64_t)(oa + ma) * nao + oc + y], kac[y]);
            if (w_ad)
#pragma unroll
                for (int y = 0; y < ND; ++y) unsafeAtomicAdd(&K[(int64_t)(oa + ma) * nao + od + y], kad[y]);
        }
        if constexpr (!S::split_a) {
            if (w_bc)
#pragma unroll
                for (int x = 0; x < NB; ++x)
#pragma unroll
                    for (int y = 0; y < NC; ++y) unsafeAtomicAdd(&K[(int64_t)(ob + x) * nao + oc + y], kbc[x][y]);
            if (w_bd)
#pragma unroll
                for (int x = 0; x < NB; ++x)
#pragma unroll
                    for (int y = 0; y < ND; ++y) unsafeAtomicAdd(&K[(int64_t)(ob + x) * nao + od + y], kbd[x][y]);
        }
    }
    if (!do_j) return;
    if constexpr (TK > 1) {
        // the TK lanes of one bra pair are adjacent: sum their Hermite J vectors
        int a = any ? 1 : 0;
#pragma unroll
        for (int w = TK / 2; w > 0; w >>= 1) {
#pragma unroll
            for (int h = 0; h < NHB; ++h) jh[h] += __shfl_xor(jh[h], w);
            a |= __shfl_xor(a, w);
        }
        any = a != 0;
    }
    if (valid && any && jk == 0) {
#pragma unroll
        for (int h = 0; h < NHB; ++h)
            unsafeAtomicAdd(&Jh[bra.herm_off + (int64_t)h * bra.npad + i], jh[h]);
    }
}

// J_f = sum_h E_f[h] Jh[h] for every pair of one class, written to both
// triangles (one triangle's positions for a = b: the block holds both).
template <int LA, int LB>
__global__ __launch_bounds__(128) void k_jout(DirectClassDev c, const double *__restrict__ Jh, int64_t nao,
                                              double *__restrict__ J)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NH = nherm(LA + LB);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    const int oa = c.off_a[i], ob = c.off_b[i];
    const bool same = c.sh_a[i] == c.sh_b[i];
    double jh[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) jh[h] = Jh[c.herm_off + (int64_t)h * c.npad + i];
#pragma unroll
    for (int ma = 0; ma < NA; ++ma)
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
            const int f = ma * NB + mb;
            double s = 0.0;
#pragma unroll
            for (int h = 0; h < NH; ++h) s += c.Eb[(int64_t)(f * NH + h) * c.npad + i] * jh[h];
            J[(int64_t)(oa + ma) * nao + ob + mb] = s;
            if (!same) J[(int64_t)(ob + mb) * nao + oa + ma] = s;
        }
}

// Symmetrise J (mean of the two triangles), complete K from its lower shell
// triangle (mean on diagonal shell blocks), add the reference J0, K0 of an
// incremental build, and form the block partials of sum D.J and sum D.K
// over the lower triangle mu >= nu.
__global__ __launch_bounds__(256) void k_direct_finish(int64_t nao, const int32_t *__restrict__ fn_shell,
                                                       const double *__restrict__ D, const double *__restrict__ J0,
                                                       const double *__restrict__ K0, double *__restrict__ J,
                                                       double *__restrict__ K, double *__restrict__ Epart)
{
    const int64_t ntri = nao * (nao + 1) / 2;
    double ej = 0.0, ek = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ntri; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t mu = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
        while (mu * (mu + 1) / 2 > e) --mu;
        while ((mu + 1) * (mu + 2) / 2 <= e) ++mu;
        const int64_t nu = e - mu * (mu + 1) / 2;
        const int64_t a = mu * nao + nu, b = nu * nao + mu;
        double jv = mu == nu ? J[a] : 0.5 * (J[a] + J[b]);
        double kv = (fn_shell[mu] == fn_shell[nu] && mu != nu) ? 0.5 * (K[a] + K[b]) : K[a];
        if (J0) { jv += J0[a]; kv += K0[a]; }   // increment on top of the reference (symmetric) J0, K0
        J[a] = jv; J[b] = jv;
        K[a] = kv; K[b] = kv;
        const double dw = mu == nu ? D[a] : D[a] + D[b];
        ej += dw * jv;
        ek += dw * kv;
    }
    __shared__ double sj[256], sk[256];
    sj[threadIdx.x] = ej; sk[threadIdx.x] = ek;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { sj[threadIdx.x] += sj[threadIdx.x + w]; sk[threadIdx.x] += sk[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { Epart[blockIdx.x] = sj[0]; Epart[256 + blockIdx.x] = sk[0]; }
}

// E_J = 1/2 sum D.J, E_K = -1/4 sum D.K from the 256 block partials, in a fixed order.
__global__ __launch_bounds__(256) void k_direct_energy(const double *__restrict__ Epart, double *__restrict__ E)
{
    __shared__ double sj[256], sk[256];
    sj[threadIdx.x] = Epart[threadIdx.x]; sk[threadIdx.x] = Epart[256 + threadIdx.x];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { sj[threadIdx.x] += sj[threadIdx.x + w]; sk[threadIdx.x] += sk[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { E[0] = 0.5 * sj[0]; E[1] = -0.25 * sk[0]; }
}

template <int LA, int LB, int LC, int LD, bool TILED>
static void launch_shape(const DirectClassDev &bra, const DirectClassDev &ket, double tau, const double *boys,
                         const double *D, int64_t nao, const double *Dh, double *Jh, double *K, const double *dsh,
                         int nsh, hipStream_t s)
{
    using S = QuartetShape<TILED, LA>;
    const int gx = (bra.n + S::TB - 1) / S::TB;
    const int gz = S::split_a ? 2 * LA + 1 : 1;
    // split the ket range into about 32768 waves per launch, at least two
    // ket pairs (or one tile step) per split: with pairs sorted by Schwarz
    // factor, short splits let the many waves whose bound fails early end
    // early, and the long loops of the leading pairs spread over the chip
    // (measured against 4096 / 8192 / 16384 waves and 4-32 pairs)
    const int minchunk = S::heavy ? S::TK : 2;
    const int want = std::max(1, (32768 + gx * gz - 1) / (gx * gz));
    const int nchunk = std::max(1, std::min(want, (ket.n + minchunk - 1) / minchunk));
    int kchunk = (ket.n + nchunk - 1) / nchunk;
    kchunk = (kchunk + S::TK - 1) / S::TK * S::TK;
    const int gy = (ket.n + kchunk - 1) / kchunk;
    hipLaunchKernelGGL((k_direct<LA, LB, LC, LD, TILED>), dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(64), 0,
                       s, bra, ket, kchunk, tau, boys, D, nao, Dh, Jh, K, 1, dsh, nsh);
}

// Tiled shape for total angular momentum 5 and up; for a d shell first in the
// bra (pairs few and costly) when that class has under 512 pairs; else plain.
template <int LA, int LB, int LC, int LD>
static void launch_quartets(const DirectClassDev &bra, const DirectClassDev &ket, double tau, const double *boys,
                            const double *D, int64_t nao, const double *Dh, double *Jh, double *K, const double *dsh,
                            int nsh, hipStream_t s)
{
    constexpr int L = LA + LB + LC + LD;
    if constexpr (L >= 5) {
        launch_shape<LA, LB, LC, LD, true>(bra, ket, tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    } else if constexpr (LA == 2) {
        if (bra.n < 512) launch_shape<LA, LB, LC, LD, true>(bra, ket, tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
        else launch_shape<LA, LB, LC, LD, false>(bra, ket, tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    } else {
        launch_shape<LA, LB, LC, LD, false>(bra, ket, tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    }
}

template <int LA, int LB>
static void launch_bra(const DirectClassDev *cls, double tau, const double *boys, const double *D, int64_t nao,
                       const double *Dh, double *Jh, double *K, const double *dsh, int nsh, hipStream_t s)
{
    const DirectClassDev &b = cls[LA == 0 ? 0 : (LA == 1 ? 1 + LB : 3 + LB)];
    if (b.n <= 0) return;
    if (cls[0].n > 0) launch_quartets<LA, LB, 0, 0>(b, cls[0], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    if (cls[1].n > 0) launch_quartets<LA, LB, 1, 0>(b, cls[1], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    if (cls[2].n > 0) launch_quartets<LA, LB, 1, 1>(b, cls[2], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    if (cls[3].n > 0) launch_quartets<LA, LB, 2, 0>(b, cls[3], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    if (cls[4].n > 0) launch_quartets<LA, LB, 2, 1>(b, cls[4], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    if (cls[5].n > 0) launch_quartets<LA, LB, 2, 2>(b, cls[5], tau, boys, D, nao, Dh, Jh, K, dsh, nsh, s);
}

template <int LA, int LB>
static void launch_pair_pass(const DirectClassDev &c, const double *D, int64_t nao, double *Dh, const double *Jh,
                             double *J, bool jout, hipStream_t s)
{
    if (c.n <= 0) return;
    const dim3 grid((unsigned)((c.n + 127) / 128));
    if (jout) hipLaunchKernelGGL((k_jout<LA, LB>), grid, dim3(128), 0, s, c, Jh, nao, J);
    else hipLaunchKernelGGL((k_dherm<LA, LB>), grid, dim3(128), 0, s, c, D, nao, Dh);
}

static void pair_passes(const DirectClassDev *cls, const double *D, int64_t nao, double *Dh, const double *Jh,
                        double *J, bool jout, hipStream_t s)
{
    launch_pair_pass<0, 0>(cls[0], D, nao, Dh, Jh, J, jout, s);
    launch_pair_pass<1, 0>(cls[1], D, nao, Dh, Jh, J, jout, s);
    launch_pair_pass<1, 1>(cls[2], D, nao, Dh, Jh, J, jout, s);
    launch_pair_pass<2, 0>(cls[3], D, nao, Dh, Jh, J, jout, s);
    launch_pair_pass<2, 1>(cls[4], D, nao, Dh, Jh, J, jout, s);
    launch_pair_pass<2, 2>(cls[5], D, nao, Dh, Jh, J, jout, s);
}

void launch_direct_build(const Plan &p, const DirectLayout &L, const double *C, int32_t nocc, const double *Din,
                         const double *D0, const double *J0, const double *K0, double *J, double *K, double *E,
                         char *scratch, hipStream_t s)
{
    const int64_t nao = p.nao;
    const DirectState &ds = p.dir;
    const double *Dfull = Din;
    if (!L.with_D) {
        double *Dw = reinterpret_cast<double *>(scratch + L.o_D);
        launch_density(C, nao, nocc, 2.0, Dw, s);
        Dfull = Dw;
    }
    // the density whose J and K are integrated: D, or dD = D - D0 with the
    // shell-block bound table of the density-weighted screen
    const double *D = Dfull;
    const double *dsh = nullptr;
    if (L.delta) {
        double *dD = reinterpret_cast<double *>(scratch + L.o_D);
        double *tab = reinterpret_cast<double *>(scratch + L.o_dsh);
        hipLaunchKernelGGL(k_dsub, dim3((unsigned)((nao * nao + 255) / 256)), dim3(256), 0, s, Din, D0, nao * nao, dD);
        const int64_t nxy = (int64_t)p.nsh_ao * p.nsh_ao;
        hipLaunchKernelGGL(k_shell_dmax, dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, s, dD, nao, p.nsh_ao,
                           ds.shell_off, tab);
        hipLaunchKernelGGL(k_dmax_all, dim3(1), dim3(256), 0, s, tab, nxy);
        D = dD;
        dsh = tab;
    }
    const int nsh = p.nsh_ao;
    double *Dh = reinterpret_cast<double *>(scratch + L.o_Dh);
    double *Jh = reinterpret_cast<double *>(scratch + L.o_Jh);
    double *Epart = reinterpret_cast<double *>(scratch + L.o_Epart);
    dfill(J, nao * nao, s);
    dfill(K, nao * nao, s);
    dfill(Jh, ds.herm_total, s);
    pair_passes(ds.cls, D, nao, Dh, nullptr, nullptr, false, s);
    const double tau = p.thresh;
    launch_bra<0, 0>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    launch_bra<1, 0>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    launch_bra<1, 1>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    launch_bra<2, 0>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    launch_bra<2, 1>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    launch_bra<2, 2>(ds.cls, tau, ds.boys, D, nao, Dh, Jh, K, dsh, nsh, s);
    pair_passes(ds.cls, D, nao, Dh, Jh, J, true, s);
    hipLaunchKernelGGL(k_direct_finish, dim3(256), dim3(256), 0, s, nao, ds.fn_shell, Dfull, L.delta ? J0 : nullptr,
                       L.delta ? K0 : nullptr, J, K, Epart);
    hipLaunchKernelGGL(k_direct_energy, dim3(1), dim3(256), 0, s, Epart, E);
}

}  // namespace dfjk
