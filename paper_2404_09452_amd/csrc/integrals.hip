// Gaussian-integral kernels for gfx950: Boys evaluation, Schwarz factors,
// three-centre (mu nu|P) and the two-centre metric (P|Q).
//
// Method (McMurchie-Davidson with a solid-harmonic ket).  The bra product of
// two AO shells is expanded in Hermite Gaussians at P with coefficients
// E^{ab}_{tuv}.  A pure solid-harmonic Gaussian S_lm(r-C) exp(-g|r-C|^2) is,
// by Hobson's theorem, exactly (2g)^{-l} sum_{tau+nu+phi=l} s_lm(tau,nu,phi)
// d^tau_Cx d^nu_Cy d^phi_Cz exp(-g|r-C|^2), so the ket needs only Hermite
// orders of total degree l and no Cartesian-to-spherical step.  Then
//   (ab|c) = N_a N_b N_c 2 pi^{5/2} / (p g sqrt(p+g)) (-1)^l (2g)^{-l}
//            sum_{tuv} E^{ab}_{tuv} sum_{|tau nu phi|=l} s_lm R_{t+tau,u+nu,v+phi}(alpha, P-C),
// alpha = p g/(p+g).  The bra is taken to spherical form after the sums.
// One thread evaluates one (shell pair, aux shell) triplet; a launch covers
// one (la, lb, lc) class so every loop is unrolled at compile time.
#include <array>
#include <vector>

#include "dfjk_internal.h"
#include "hermite.h"

namespace dfjk {

// Solid-harmonic monomial coefficients and the Boys Taylor table; one copy per
// device, written once by ensure_device_constants.
__constant__ double c_sph[kMaxLAux + 1][7][10];
__device__ double g_boys[kBoysNT * kBoysNM];

void upload_constants(const double coef[kMaxLAux + 1][7][10], hipStream_t s)
{
    (void)s;
    (void)hipMemcpyToSymbol(HIP_SYMBOL(c_sph), coef, sizeof(double) * (kMaxLAux + 1) * 70, 0,
                            hipMemcpyHostToDevice);
}

void upload_boys_table(const double *host, size_t n, const double **dev_addr, hipError_t *err)
{
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_boys), host, n * sizeof(double), 0, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_boys));
        *dev_addr = static_cast<const double *>(ptr);
    }
    *err = e;
}

// --------------------------------------------------------------------------
// Boys function on an array (tests the device routine the kernels use).

template <int M>
__global__ void k_boys_eval(int64_t n, const double *__restrict__ T, double *__restrict__ F,
                            const double *__restrict__ tab)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = T[i];
    if (!(t >= 0.0) || !(t < 1e300)) {   // negative, NaN or infinite: no table lookup
#pragma unroll
        for (int m = 0; m <= M; ++m) F[i * (M + 1) + m] = __builtin_nan("");
        return;
    }
    double f[M + 1];
    boys<M>(t, f, tab);
#pragma unroll
    for (int m = 0; m <= M; ++m) F[i * (M + 1) + m] = f[m];
}

void launch_boys_eval(int mmax, int64_t n, const double *T, double *F, const double *tab, hipStream_t s)
{
    const int bs = 256;
    const unsigned nb = (unsigned)((n + bs - 1) / bs);
#define BOYS_CASE(M) \
    case M: hipLaunchKernelGGL(k_boys_eval<M>, dim3(nb), dim3(bs), 0, s, n, T, F, tab); break;
    switch (mmax) {
        BOYS_CASE(0) BOYS_CASE(1) BOYS_CASE(2) BOYS_CASE(3) BOYS_CASE(4) BOYS_CASE(5)
        BOYS_CASE(6) BOYS_CASE(7) BOYS_CASE(8) BOYS_CASE(9) BOYS_CASE(10) BOYS_CASE(11)
        BOYS_CASE(12) BOYS_CASE(13) BOYS_CASE(14) BOYS_CASE(15) BOYS_CASE(16)
    }
#undef BOYS_CASE
}

// --------------------------------------------------------------------------
// Schwarz factors.  At coincident centres R_{tuv}(alpha, 0) vanishes unless
// t, u, v are all even, and R_{2i,2j,2k} = (2i-1)!!(2j-1)!!(2k-1)!!
// (-2 alpha)^{i+j+k} / (2(i+j+k)+1).

constexpr double dfact_m1(int n)   // (n-1)!! for even n, (−1)!! = 1
{
    double r = 1.0;
    for (int k = n - 1; k > 1; k -= 2) r *= k;
    return r;
}

template <int L>
__device__ __forceinline__ void hermite_R_origin(double alpha, double (&R)[nherm(L)])
{
    double pw[L / 2 + 1];
    pw[0] = 1.0;
#pragma unroll
    for (int s = 1; s <= L / 2; ++s) pw[s] = pw[s - 1] * (-2.0 * alpha);
#pragma unroll
    for (int t = 0; t <= L; ++t)
#pragma unroll
        for (int u = 0; u + t <= L; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= L; ++v) {
                if ((t | u | v) & 1) {
                    R[hidx(t, u, v)] = 0.0;
                } else {
                    const int s = (t + u + v) / 2;
                    R[hidx(t, u, v)] = dfact_m1(t) * dfact_m1(u) * dfact_m1(v) * pw[s] / (2 * s + 1);
                }
            }
}

// Spherical-bra Hermite coefficients of function pair (ma, mb):
// Es[tuv] = sum_{ca,cb} s_a[ma][ca] s_b[mb][cb] Ex Ey Ez.
template <int LA, int LB>
__device__ __forceinline__ void bra_sph(int ma, int mb, const double (&Ex)[LA + 1][LB + 1][LA + LB + 1],
                                        const double (&Ey)[LA + 1][LB + 1][LA + LB + 1],
                                        const double (&Ez)[LA + 1][LB + 1][LA + LB + 1],
                                        double (&Es)[nherm(LA + LB)])
{
    constexpr int CA = ncart(LA), CB = ncart(LB);
#pragma unroll
    for (int i = 0; i < nherm(LA + LB); ++i) Es[i] = 0.0;
#pragma unroll
    for (int ca = 0; ca < CA; ++ca) {
        const double sa = c_sph[LA][ma][ca];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const double s = sa * c_sph[LB][mb][cb];
            const int ax = cart_pow(LA, ca, 0), ay = cart_pow(LA, ca, 1), az = cart_pow(LA, ca, 2);
            const int bx = cart_pow(LB, cb, 0), by = cart_pow(LB, cb, 1), bz = cart_pow(LB, cb, 2);
#pragma unroll
            for (int t = 0; t <= ax + bx; ++t)
#pragma unroll
                for (int u = 0; u <= ay + by; ++u)
#pragma unroll
                    for (int v = 0; v <= az + bz; ++v)
                        Es[hidx(t, u, v)] += s * Ex[ax][bx][t] * Ey[ay][by][u] * Ez[az][bz][v];
        }
    }
}

// R_{tuv}(alpha, 0) / (-2 alpha)^{(t+u+v)/2} for even t, u, v (zero otherwise):
// (t-1)!! (u-1)!! (v-1)!! / (t+u+v+1), a compile-time constant.
constexpr double kDfactM1[9] = {1.0, 0.0, 1.0, 0.0, 3.0, 0.0, 15.0, 0.0, 105.0};   // (n-1)!!, even n
constexpr double r_origin_coef(int t, int u, int v)
{
    return ((t | u | v) & 1) ? 0.0 : kDfactM1[t] * kDfactM1[u] * kDfactM1[v] / (t + u + v + 1);
}

// sqrt(|(ab|ab)|) of one function pair from its spherical bra Es: the bra
// twice, the ket's Hermite signs (-1)^{t'+u'+v'} and R at coincident centres
// (alpha = p/2).
template <int LAB>
__device__ __forceinline__ double schwarz_form(const double (&Es)[nherm(LAB)], double p, double na, double nb)
{
    double pw[LAB + 1];   // (-2 alpha)^s
    pw[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= LAB; ++k) pw[k] = pw[k - 1] * (-p);
    double s = 0.0;
#pragma unroll
    for (int t = 0; t <= LAB; ++t)
#pragma unroll
        for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= LAB; ++v) {
                double inner = 0.0;
#pragma unroll
                for (int t2 = 0; t2 <= LAB; ++t2)
#pragma unroll
                    for (int u2 = 0; u2 + t2 <= LAB; ++u2)
#pragma unroll
                        for (int v2 = 0; v2 + u2 + t2 <= LAB; ++v2) {
                            if (((t + t2) | (u + u2) | (v + v2)) & 1) continue;
                            const double c = (((t2 + u2 + v2) & 1) ? -1.0 : 1.0) *
                                             r_origin_coef(t + t2, u + u2, v + v2);
                            inner += (c * pw[(t + t2 + u + u2 + v + v2) / 2]) * Es[hidx(t2, u2, v2)];
                        }
                s += Es[hidx(t, u, v)] * inner;
            }
    const double pref = kTwoPi52 / (p * p * sqrt(2.0 * p)) * (na * nb) * (na * nb);
    return sqrt(fabs(s) * pref);
}

// Largest sqrt|(ab|ab)| over the function pairs of one shell pair (classes
// below (d d)): the Hermite tables once, then each function pair's bra.
template <int LA, int LB>
__device__ double schwarz_pair_max(double ea, double eb, double ax_, double ay_, double az_, double bx_, double by_,
                                   double bz_, double na, double nb)
{
    constexpr int LAB = LA + LB, NB = 2 * LB + 1;
    const double p = ea + eb, ip = 1.0 / p;
    const double Px = (ea * ax_ + eb * bx_) * ip, Py = (ea * ay_ + eb * by_) * ip,
                 Pz = (ea * az_ + eb * bz_) * ip;
    const double mu = ea * eb * ip;
    double Ex[LA + 1][LB + 1][LAB + 1], Ey[LA + 1][LB + 1][LAB + 1], Ez[LA + 1][LB + 1][LAB + 1];
    hermite_E<LA, LB>(Px - ax_, Px - bx_, 0.5 * ip, exp(-mu * (ax_ - bx_) * (ax_ - bx_)), Ex);
    hermite_E<LA, LB>(Py - ay_, Py - by_, 0.5 * ip, exp(-mu * (ay_ - by_) * (ay_ - by_)), Ey);
    hermite_E<LA, LB>(Pz - az_, Pz - bz_, 0.5 * ip, exp(-mu * (az_ - bz_) * (az_ - bz_)), Ez);
    double best = 0.0;
#pragma unroll 1
    for (int k = 0; k < (2 * LA + 1) * NB; ++k) {
        double Es[nherm(LAB)];
        bra_sph<LA, LB>(k / NB, k % NB, Ex, Ey, Ez, Es);
        best = fmax(best, schwarz_form<LAB>(Es, p, na, nb));
    }
    return best;
}

// Schwarz factor of every shell pair a >= b other than (d d): the largest
// (ab|ab) over its function pairs, one thread per pair; (d d) pairs get 0
// here and their value from k_schwarz_dd.
__global__ __launch_bounds__(256) void k_schwarz_pairs(int64_t npair, ShellsDev ao, double *__restrict__ q)
{
    const int64_t ab = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (ab >= npair) return;
    int a = (int)((sqrt(8.0 * (double)ab + 1.0) - 1.0) * 0.5);
    while ((int64_t)a * (a + 1) / 2 > ab) --a;
    while ((int64_t)(a + 1) * (a + 2) / 2 <= ab) ++a;
    int b = (int)(ab - (int64_t)a * (a + 1) / 2);
    if (ao.l[a] < ao.l[b]) { const int t = a; a = b; b = t; }
    const int la = ao.l[a], lb = ao.l[b];
    double r = 0.0;
#define SCH(LA, LB)                                                                                   \
    r = schwarz_pair_max<LA, LB>(ao.exp[a], ao.exp[b], ao.x[a], ao.y[a], ao.z[a], ao.x[b], ao.y[b], \
                                 ao.z[b], ao.norm[a], ao.norm[b]);
    if (la == 0) { SCH(0, 0) }
    else if (la == 1) { if (lb == 0) { SCH(1, 0) } else { SCH(1, 1) } }
    else if (lb == 0) { SCH(2, 0) }
    else if (lb == 1) { SCH(2, 1) }
#undef SCH
    q[ab] = r;
}

// (d d) pairs: pair (i >= j) of the ascending d-shell list dsh, 32 lanes per
// pair, lane k < 25 taking function pair k.  Lane 0 forms the three Hermite
// tables into LDS, each lane builds its bra from them, and the largest value
// is kept with an integer maximum on the bits (non-negative values order as
// their bit patterns do) in q, which k_schwarz_pairs has set to 0.
__global__ __launch_bounds__(256) void k_schwarz_dd(int64_t ndd, const int32_t *__restrict__ dsh, ShellsDev ao,
                                                    double *__restrict__ q)
{
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t ij = gid >> 5;
    const int k = (int)(gid & 31);
    if (ij >= ndd || k >= 25) return;
    int i = (int)((sqrt(8.0 * (double)ij + 1.0) - 1.0) * 0.5);
    while ((int64_t)i * (i + 1) / 2 > ij) --i;
    while ((int64_t)(i + 1) * (i + 2) / 2 <= ij) ++i;
    const int j = (int)(ij - (int64_t)i * (i + 1) / 2);
    const int a = dsh[i], b = dsh[j];
    __shared__ double tab[8][3][3][3][5];
    double (&T)[3][3][3][5] = tab[threadIdx.x >> 5];
    const double ea = ao.exp[a], eb = ao.exp[b];
    const double p = ea + eb, ip = 1.0 / p;
    if (k == 0) {
        const double A[3] = {ao.x[a], ao.y[a], ao.z[a]}, B[3] = {ao.x[b], ao.y[b], ao.z[b]};
        const double mu = ea * eb * ip;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double P = (ea * A[d] + eb * B[d]) * ip;
            double E[3][3][5];
            hermite_E<2, 2>(P - A[d], P - B[d], 0.5 * ip, exp(-mu * (A[d] - B[d]) * (A[d] - B[d])), E);
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
                for (int y = 0; y < 3; ++y)
#pragma unroll
                    for (int t = 0; t <= x + y; ++t) T[d][x][y][t] = E[x][y][t];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int ma = k / 5, mb = k % 5;
    double Es[nherm(4)];
#pragma unroll
    for (int h = 0; h < nherm(4); ++h) Es[h] = 0.0;
#pragma unroll
    for (int ca = 0; ca < 6; ++ca) {
        const double sa = c_sph[2][ma][ca];
#pragma unroll
        for (int cb = 0; cb < 6; ++cb) {
            const double sab = sa * c_sph[2][mb][cb];
            const int ax = cart_pow(2, ca, 0), ay = cart_pow(2, ca, 1), az = cart_pow(2, ca, 2);
            const int bx = cart_pow(2, cb, 0), by = cart_pow(2, cb, 1), bz = cart_pow(2, cb, 2);
#pragma unroll
            for (int t = 0; t <= ax + bx; ++t)
#pragma unroll
                for (int u = 0; u <= ay + by; ++u) {
                    const double xy = sab * T[0][ax][bx][t] * T[1][ay][by][u];
#pragma unroll
                    for (int v = 0; v <= az + bz; ++v) Es[hidx(t, u, v)] += xy * T[2][az][bz][v];
                }
        }
    }
    const double r = schwarz_form<4>(Es, p, ao.norm[a], ao.norm[b]);
    const int64_t ab = (int64_t)a * (a + 1) / 2 + b;
    atomicMax(reinterpret_cast<unsigned long long *>(q) + ab, (unsigned long long)__double_as_longlong(r));
}

// dsh: the nd d shells in ascending order (device memory)
void launch_schwarz_pairs(int64_t npair, const ShellsDev &ao, const int32_t *dsh, int32_t nd, double *q,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_schwarz_pairs, dim3((unsigned)((npair + 255) / 256)), dim3(256), 0, s, npair, ao, q);
    const int64_t ndd = (int64_t)nd * (nd + 1) / 2;
    if (ndd > 0)
        hipLaunchKernelGGL(k_schwarz_dd, dim3((unsigned)((ndd * 32 + 255) / 256)), dim3(256), 0, s, ndd, dsh, ao, q);
}

// (c|c) of one solid-harmonic Gaussian, largest over m (all equal in exact
// arithmetic by rotational invariance of the Coulomb operator).
template <int LC>
__device__ double schwarz_aux(double g, double nc)
{
    constexpr int CC = ncart(LC), L = 2 * LC;
    double R[nherm(L)];
    hermite_R_origin<L>(0.5 * g, R);
    double scale = 1.0;
    for (int k = 0; k < LC; ++k) scale /= (2.0 * g) * (2.0 * g);
    const double pref = kTwoPi52 / (g * g * sqrt(2.0 * g)) * nc * nc * scale * ((LC & 1) ? -1.0 : 1.0);
    double best = 0.0;
    for (int m = 0; m < 2 * LC + 1; ++m) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < CC; ++i)
#pragma unroll
            for (int j = 0; j < CC; ++j) {
                const int t = cart_pow(LC, i, 0) + cart_pow(LC, j, 0);
                const int u = cart_pow(LC, i, 1) + cart_pow(LC, j, 1);
                const int v = cart_pow(LC, i, 2) + cart_pow(LC, j, 2);
                s += c_sph[LC][m][i] * c_sph[LC][m][j] * R[hidx(t, u, v)];
            }
        best = fmax(best, fabs(s * pref));
    }
    return sqrt(best);
}

__global__ void k_schwarz_aux(int32_t nsh, ShellsDev ax, double *__restrict__ q)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nsh) return;
    const double g = ax.exp[c], nc = ax.norm[c];
    double r;
    switch (ax.l[c]) {
    case 0: r = schwarz_aux<0>(g, nc); break;
    case 1: r = schwarz_aux<1>(g, nc); break;
    case 2: r = schwarz_aux<2>(g, nc); break;
    default: r = schwarz_aux<3>(g, nc); break;
    }
    q[c] = r;
}

void launch_schwarz_aux(int32_t nsh, const ShellsDev &ax, double *q, hipStream_t s)
{
    const int bs = 128;
    hipLaunchKernelGGL(k_schwarz_aux, dim3((nsh + bs - 1) / bs), dim3(bs), 0, s, nsh, ax, q);
}

// --------------------------------------------------------------------------
// Three-centre integrals.
//
// Work split.  Everything that depends only on the shell pair (a, b) is formed
// once per pair by k_pair_rec: the Gaussian product p, P and the spherical bra
// Hermite coefficients
//   Eh[tuv][ab] = 2 pi^{5/2} N_a N_b / p * t! u! v! * sum_{ca,cb} s_a s_b E^x E^y E^z.
// k_int3c then gives each lane one output column, an (aux shell c, m_c)
// combination: floor(64 / (2 lc + 1)) aux shells per wave, all m_c of a shell in
// adjacent lanes, so a row (a function pair) is stored as one contiguous run.
// The pair record is the same for the whole wave and is read through scalar
// loads, so the bra contraction takes its coefficient as a scalar operand.
//
// Ket by Hobson's theorem applied a second time.  With G = F_lc(alpha r^2),
//   sum_k s_m(k) R_{tuv+k} = d^{tuv}[S_m(X, Y, Z) (-2 alpha)^lc G],
// the derivative of a harmonic polynomial times a radial function (S_m(grad)
// of a function of r^2 is S_m(r) (2 d/dr^2)^lc of it).  By Leibniz, with
// Taylor-scaled factors D[d] = d^d S_m / d! and G'[tuv] = d^{tuv} G / tuv!,
//   W'[tuv] = sum_{d <= tuv, |d| <= lc} D[d] G'[tuv - d]   (= W[tuv] / tuv!),
// so a lane holds the Hermite table only up to the bra order la + lb instead of
// la + lb + lc, and (ab|c m) = N_c (alpha/g)^lc / (g sqrt(p+g)) sum_tuv Eh[tuv][ab] W'[tuv]
// (the ket factor (-1/(2g))^lc times (-2 alpha)^lc).

struct Int3cArgs {
    const int32_t *pa, *pb, *pf0;
    const double *pq;
    int32_t p_begin, p_end, c_begin, c_end;
    ShellsDev ao, ax;
    const double *boys;
    double tau;
    const double *rec;        // record of pair rec_first of this class
    int32_t rec_first;
    double *U;                // rows f - f_base (a block of function-pair rows)
    int64_t ld;
    int64_t f_base;
};

constexpr double kFact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
constexpr double kInvFact[5] = {1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0};

// Terms of D[d] = sum_{|k| = l, k >= d} s(k) C(kx,dx) C(ky,dy) C(kz,dz) X^{kx-dx} Y^{ky-dy} Z^{kz-dz}:
// Hermite index of d, Cartesian index of k, monomial index of k - d, binomial factor.
template <int LC>
struct KetTerms {
    int n;
    int d[64], k[64], m[64];
    double c[64];
};
template <int LC>
constexpr KetTerms<LC> ket_terms()
{
    KetTerms<LC> t{};
    constexpr double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    int k = 0;
    for (int kx = LC; kx >= 0; --kx)
        for (int ky = LC - kx; ky >= 0; --ky, ++k) {
            const int kz = LC - kx - ky;
            for (int dx = 0; dx <= kx; ++dx)
                for (int dy = 0; dy <= ky; ++dy)
                    for (int dz = 0; dz <= kz; ++dz) {
                        t.d[t.n] = hidx(dx, dy, dz);
                        t.k[t.n] = k;
                        t.m[t.n] = hidx(kx - dx, ky - dy, kz - dz);
                        t.c[t.n] = binom[kx][dx] * binom[ky][dy] * binom[kz][dz];
                        ++t.n;
                    }
        }
    return t;
}

// One thread per (pair, ma, mb) of the class's pairs p_begin..p_end (records
// from rec, in pair order).
template <int LA, int LB>
__device__ __forceinline__ void pair_rec(const Int3cArgs &g, double *__restrict__ rec, int64_t tid)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NAB = NA * NB, LAB = LA + LB;
    constexpr int RS = pair_rec_doubles(LA, LB);
    if (tid >= (int64_t)(g.p_end - g.p_begin) * NAB) return;
    const int pl = (int)(tid / NAB), ab = (int)(tid % NAB);
    const int ip = g.p_begin + pl;
    const int a = g.pa[ip], b = g.pb[ip];
    const double ea = g.ao.exp[a], eb = g.ao.exp[b];
    const double Ax = g.ao.x[a], Ay = g.ao.y[a], Az = g.ao.z[a];
    const double Bx = g.ao.x[b], By = g.ao.y[b], Bz = g.ao.z[b];
    const double p = ea + eb, ipp = 1.0 / p;
    const double Px = (ea * Ax + eb * Bx) * ipp, Py = (ea * Ay + eb * By) * ipp, Pz = (ea * Az + eb * Bz) * ipp;
    const double mu = ea * eb * ipp;
    double Ex[LA + 1][LB + 1][LAB + 1], Ey[LA + 1][LB + 1][LAB + 1], Ez[LA + 1][LB + 1][LAB + 1];
    hermite_E<LA, LB>(Px - Ax, Px - Bx, 0.5 * ipp, exp(-mu * (Ax - Bx) * (Ax - Bx)), Ex);
    hermite_E<LA, LB>(Py - Ay, Py - By, 0.5 * ipp, exp(-mu * (Ay - By) * (Ay - By)), Ey);
    hermite_E<LA, LB>(Pz - Az, Pz - Bz, 0.5 * ipp, exp(-mu * (Az - Bz) * (Az - Bz)), Ez);
    double Es[nherm(LAB)];
    bra_sph<LA, LB>(ab / NB, ab % NB, Ex, Ey, Ez, Es);
    double *r = rec + (int64_t)pl * RS;
    if (ab == 0) {
        r[0] = p; r[1] = Px; r[2] = Py; r[3] = Pz; r[4] = g.pq[ip]; r[5] = 0.0; r[6] = 0.0; r[7] = 0.0;
    }
    const double pref = kTwoPi52 * ipp * g.ao.norm[a] * g.ao.norm[b];
#pragma unroll
    for (int t = 0; t <= LAB; ++t)
#pragma unroll
        for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= LAB; ++v)
                r[8 + hidx(t, u, v) * NAB + ab] = pref * (kFact[t] * kFact[u] * kFact[v]) * Es[hidx(t, u, v)];
}

template <int LA, int LB>
__global__ __launch_bounds__(256) void k_pair_rec(Int3cArgs g, double *__restrict__ rec)
{
    pair_rec<LA, LB>(g, rec, blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
}

// The pair records of one class for several molecules in one launch
// (workgroup b belongs to molecule m for blk_start[m] <= b < blk_start[m+1]).
constexpr int kPairRecGroupMax = 14;
struct PairRecGroup {
    int32_t n;
    uint32_t blk_start[kPairRecGroupMax + 1];
    double *rec[kPairRecGroupMax];
    Int3cArgs g[kPairRecGroupMax];
};
static_assert(sizeof(PairRecGroup) <= 4096, "kernel arguments are limited to 4 KB");

template <int LA, int LB>
__global__ __launch_bounds__(256) void k_pair_rec_group(PairRecGroup grp)
{
    int m = 0;
    while (m + 1 < grp.n && blockIdx.x >= grp.blk_start[m + 1]) ++m;
    pair_rec<LA, LB>(grp.g[m], grp.rec[m], (blockIdx.x - grp.blk_start[m]) * (int64_t)blockDim.x + threadIdx.x);
}

// Shared pieces of both lane layouts: the Taylor-scaled Hermite table G' of
// F_lc(alpha r^2) to the bra order, the monomials of (X, Y, Z) to order lc,
// the ket factor D of one m_c, and the bra contraction.
template <int LAB, int LC>
__device__ __forceinline__ void ket_table(double p, double X, double Y, double Z, double gc, const double *boys_tab,
                                          double (&G)[nherm(LAB)], double (&M)[nherm(LC)], double &scale)
{
    constexpr int L = LAB + LC;
    const double pg = p + gc, ipg = 1.0 / pg;
    const double alpha = p * gc * ipg;
    double F[L + 1];
    boys<L>(alpha * (X * X + Y * Y + Z * Z), F, boys_tab);
    hermite_R<LAB, LC>(alpha, X, Y, Z, F, G);
#pragma unroll
    for (int t = 0; t <= LAB; ++t)
#pragma unroll
        for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= LAB; ++v) G[hidx(t, u, v)] *= kInvFact[t] * kInvFact[u] * kInvFact[v];
    double px[LC + 1], py[LC + 1], pz[LC + 1];
    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
    for (int i = 1; i <= LC; ++i) { px[i] = px[i - 1] * X; py[i] = py[i - 1] * Y; pz[i] = pz[i - 1] * Z; }
#pragma unroll
    for (int i = 0; i <= LC; ++i)
#pragma unroll
        for (int j = 0; i + j <= LC; ++j)
#pragma unroll
            for (int k = 0; i + j + k <= LC; ++k) M[hidx(i, j, k)] = px[i] * py[j] * pz[k];
    // (alpha/g)^lc / (g sqrt(p+g)); the caller multiplies in N_c
    scale = sqrt(ipg) / gc;
#pragma unroll
    for (int k = 0; k < LC; ++k) scale *= p * ipg;
}

template <int LC>
__device__ __forceinline__ void ket_factor(const double (&sv)[ncart(LC)], const double (&M)[nherm(LC)],
                                           double (&D)[nherm(LC)])
{
#pragma unroll
    for (int i = 0; i < nherm(LC); ++i) D[i] = 0.0;
    constexpr KetTerms<LC> kt = ket_terms<LC>();
#pragma unroll
    for (int i = 0; i < kt.n; ++i) D[kt.d[i]] += (kt.c[i] * sv[kt.k[i]]) * M[kt.m[i]];
}

// acc[ab] += sum_tuv e[tuv][ab] W'[tuv], W'[tuv] = sum_d D[d] G'[tuv - d]
template <int LAB, int LC, int NAB>
__device__ __forceinline__ void bra_contract(const double *__restrict__ e, const double (&D)[nherm(LC)],
                                             const double (&G)[nherm(LAB)], double (&acc)[NAB])
{
#pragma unroll
    for (int t = 0; t <= LAB; ++t)
#pragma unroll
        for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
            for (int v = 0; v + u + t <= LAB; ++v) {
                double w = 0.0;
#pragma unroll
                for (int dx = 0; dx <= t && dx <= LC; ++dx)
#pragma unroll
                    for (int dy = 0; dy <= u && dx + dy <= LC; ++dy)
#pragma unroll
                        for (int dz = 0; dz <= v && dx + dy + dz <= LC; ++dz)
                            w += D[hidx(dx, dy, dz)] * G[hidx(t - dx, u - dy, v - dz)];
                const double *eh = e + hidx(t, u, v) * NAB;
#pragma unroll
                for (int i = 0; i < NAB; ++i) acc[i] += eh[i] * w;
            }
}

// Lane per (aux shell, m_c): floor(64 / (2 lc + 1)) shells per wave, all m_c of
// a shell in adjacent lanes, so every function-pair row is stored as one
// contiguous run per wave.
template <int LA, int LB, int LC>
__device__ __forceinline__ void int3c_cols(const Int3cArgs &g, unsigned blk)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NC = 2 * LC + 1, NAB = NA * NB;
    constexpr int CC = ncart(LC), LAB = LA + LB;
    constexpr int SPW = 64 / NC, SPB = 4 * SPW;   // aux shells per wave, per workgroup
    constexpr int RS = pair_rec_doubles(LA, LB);
    const int nsc = g.c_end - g.c_begin;
    const int ngrp = (nsc + SPB - 1) / SPB;
    const int pl = (int)(blk / ngrp), grp = (int)(blk % ngrp);
    const int ip = g.p_begin + pl;
    const double *__restrict__ rec = g.rec + (int64_t)(ip - g.rec_first) * RS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sl = lane / NC, mc = lane - sl * NC;
    const int cl = grp * SPB + wave * SPW + sl;
    if (sl >= SPW || cl >= nsc) return;
    const int ic = g.c_begin + cl;
    double acc[NAB];
#pragma unroll
    for (int i = 0; i < NAB; ++i) acc[i] = 0.0;
    if (rec[4] * g.ax.q[ic] >= g.tau) {
        double G[nherm(LAB)], M[nherm(LC)], sc;
        ket_table<LAB, LC>(rec[0], rec[1] - g.ax.x[ic], rec[2] - g.ax.y[ic], rec[3] - g.ax.z[ic], g.ax.exp[ic],
                           g.boys, G, M, sc);
        double sv[CC], D[nherm(LC)];
#pragma unroll
        for (int k = 0; k < CC; ++k) sv[k] = c_sph[LC][mc][k];
        ket_factor<LC>(sv, M, D);
        bra_contract<LAB, LC, NAB>(rec + 8, D, G, acc);
        sc *= g.ax.norm[ic];
#pragma unroll
        for (int i = 0; i < NAB; ++i) acc[i] *= sc;
    }
    double *out = g.U + ((int64_t)g.pf0[ip] - g.f_base) * g.ld + g.ax.off[ic] + mc;
#pragma unroll
    for (int i = 0; i < NAB; ++i) out[i * g.ld] = acc[i];
}

template <int LA, int LB, int LC>
__global__ __launch_bounds__(256) void k_int3c(Int3cArgs g)
{
    int3c_cols<LA, LB, LC>(g, blockIdx.x);
}

// Lane per aux shell (classes with few outputs per triplet): the Boys
// function, the Hermite table and the divisions are formed once per triplet
// rather than once per m_c, every m_c is accumulated in registers, and each
// function-pair row of the wave's 64 shells goes out through LDS as one
// contiguous run of 64 (2 lc + 1) values.
// buf: 4 x 64 (2 lc + 1) doubles of LDS, one run per wave.
template <int LA, int LB, int LC>
__device__ __forceinline__ void int3c_shells(const Int3cArgs &g, unsigned blk, double *buf)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NC = 2 * LC + 1, NAB = NA * NB;
    constexpr int CC = ncart(LC), LAB = LA + LB;
    constexpr int RS = pair_rec_doubles(LA, LB);
    const int nsc = g.c_end - g.c_begin;
    const int ngrp = (nsc + 255) / 256;
    const int pl = (int)(blk / ngrp), grp = (int)(blk % ngrp);
    const int ip = g.p_begin + pl;
    const double *__restrict__ rec = g.rec + (int64_t)(ip - g.rec_first) * RS;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = grp * 256 + wave * 64;
    if (c0 >= nsc) return;   // whole wave past the class
    const int nv = min(64, nsc - c0);
    const int ic = g.c_begin + c0 + min(lane, nv - 1);
    double acc[NC][NAB];
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
        for (int i = 0; i < NAB; ++i) acc[m][i] = 0.0;
    if (lane < nv && rec[4] * g.ax.q[ic] >= g.tau) {
        double G[nherm(LAB)], M[nherm(LC)], sc;
        ket_table<LAB, LC>(rec[0], rec[1] - g.ax.x[ic], rec[2] - g.ax.y[ic], rec[3] - g.ax.z[ic], g.ax.exp[ic],
                           g.boys, G, M, sc);
        sc *= g.ax.norm[ic];
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            double sv[CC], D[nherm(LC)];
#pragma unroll
            for (int k = 0; k < CC; ++k) sv[k] = c_sph[LC][m][k];
            ket_factor<LC>(sv, M, D);
            bra_contract<LAB, LC, NAB>(rec + 8, D, G, acc[m]);
#pragma unroll
            for (int i = 0; i < NAB; ++i) acc[m][i] *= sc;
        }
    }
    double *row = g.U + ((int64_t)g.pf0[ip] - g.f_base) * g.ld + g.ax.off[g.c_begin + c0];
    double *b = buf + wave * 64 * NC;
#pragma unroll
    for (int i = 0; i < NAB; ++i) {
#pragma unroll
        for (int m = 0; m < NC; ++m) b[lane * NC + m] = acc[m][i];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int e = j * 64 + lane;
            if (e < nv * NC) row[i * g.ld + e] = b[e];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <int LA, int LB, int LC>
__global__ __launch_bounds__(256) void k_int3c_sh(Int3cArgs g)
{
    __shared__ double buf[4 * 64 * (2 * LC + 1)];
    int3c_shells<LA, LB, LC>(g, blockIdx.x, buf);
}

template <int LA, int LB>
static void launch_pair_class(Int3cArgs g, double *rec, hipStream_t s)
{
    constexpr int NAB = (2 * LA + 1) * (2 * LB + 1);
    const int64_t n = (int64_t)(g.p_end - g.p_begin) * NAB;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_pair_rec<LA, LB>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rec);
}

// Lane per aux shell while the outputs of a triplet, (2la+1)(2lb+1)(2lc+1),
// fit in registers beside the tables and the wave's pass over the pair record
// per m_c stays short; lane per (aux shell, m_c) otherwise (chosen per class
// from kernel times on the 128-water cluster).
constexpr bool shell_lanes_for(int la, int lb, int lc)
{
    const int nout = (2 * la + 1) * (2 * lb + 1) * (2 * lc + 1);
    const int nh = (la + lb + 1) * (la + lb + 2) * (la + lb + 3) / 6;
    return nout <= 45 && nout * nh <= 500;
}

template <int LA, int LB, int LC>
static void launch_class(Int3cArgs g, hipStream_t s)
{
    constexpr bool shell_lanes = shell_lanes_for(LA, LB, LC);
    constexpr int SPB = shell_lanes ? 256 : 4 * (64 / (2 * LC + 1));
    const int64_t npl = g.p_end - g.p_begin, nsc = g.c_end - g.c_begin;
    if (npl <= 0 || nsc <= 0) return;
    const int64_t nblk = npl * ((nsc + SPB - 1) / SPB);
    if constexpr (shell_lanes)
        hipLaunchKernelGGL((k_int3c_sh<LA, LB, LC>), dim3((unsigned)nblk), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_int3c<LA, LB, LC>), dim3((unsigned)nblk), dim3(256), 0, s, g);
}

// Several molecules' triplets of one class in one launch: workgroup b runs
// block b - blk_start[m] of molecule m (blk_start ascending), with that
// molecule's arguments, so uneven molecules share the launch.  Descriptors
// by value in the kernel arguments (no device table: the launch can be
// captured).  Every element is the same computation as in a launch of its
// own molecule, so the integrals are bitwise those of separate setups.
constexpr int kInt3cGroupMax = 16;
struct Int3cGroup {
    int32_t n;
    uint32_t blk_start[kInt3cGroupMax + 1];
    Int3cArgs g[kInt3cGroupMax];
};
static_assert(sizeof(Int3cGroup) <= 4096, "kernel arguments are limited to 4 KB");

template <int LA, int LB, int LC>
__global__ __launch_bounds__(256) void k_int3c_group(Int3cGroup grp)
{
    int m = 0;
    while (m + 1 < grp.n && blockIdx.x >= grp.blk_start[m + 1]) ++m;
    const unsigned blk = blockIdx.x - grp.blk_start[m];
    if constexpr (shell_lanes_for(LA, LB, LC)) {
        __shared__ double buf[4 * 64 * (2 * LC + 1)];
        int3c_shells<LA, LB, LC>(grp.g[m], blk, buf);
    } else {
        int3c_cols<LA, LB, LC>(grp.g[m], blk);
    }
}

// Workgroups of one molecule's launch of the class (as launch_class).
template <int LA, int LB, int LC>
static int64_t class_blocks(const Int3cArgs &g)
{
    constexpr int SPB = shell_lanes_for(LA, LB, LC) ? 256 : 4 * (64 / (2 * LC + 1));
    const int64_t npl = g.p_end - g.p_begin, nsc = g.c_end - g.c_begin;
    if (npl <= 0 || nsc <= 0) return 0;
    return npl * ((nsc + SPB - 1) / SPB);
}

template <int LA, int LB, int LC>
static void launch_class_group(const Int3cArgs *args, int n, hipStream_t s)
{
    Int3cGroup grp{};
    int64_t total = 0;
    auto flush = [&]() {
        if (grp.n == 0) return;
        grp.blk_start[grp.n] = (uint32_t)total;
        hipLaunchKernelGGL((k_int3c_group<LA, LB, LC>), dim3((unsigned)total), dim3(256), 0, s, grp);
        grp = Int3cGroup{};
        total = 0;
    };
    for (int i = 0; i < n; ++i) {
        const int64_t nb = class_blocks<LA, LB, LC>(args[i]);
        if (nb == 0) continue;
        if (grp.n == kInt3cGroupMax || total + nb > (int64_t)UINT32_MAX / 2) flush();
        grp.blk_start[grp.n] = (uint32_t)total;
        grp.g[grp.n++] = args[i];
        total += nb;
    }
    flush();
}

static ShellsDev ao_view(const Plan &p)
{
    return ShellsDev{p.d.ao_exp, p.d.ao_x, p.d.ao_y, p.d.ao_z, p.d.ao_norm, nullptr, p.d.ao_l, p.d.ao_off};
}
static ShellsDev ax_view(const Plan &p)
{
    return ShellsDev{p.d.ax_exp, p.d.ax_x, p.d.ax_y, p.d.ax_z, p.d.ax_norm, p.d.ax_q, p.d.ax_l, p.d.ax_off};
}

void pair_rec_offsets(const Plan &p, int64_t off[7])
{
    off[0] = 0;
    for (int pc = 0; pc < 6; ++pc)
        off[pc + 1] = off[pc] + (int64_t)(p.sp_class[pc].end - p.sp_class[pc].begin) *
                                    pair_rec_doubles(kPairClassLa[pc], kPairClassLb[pc]);
}

static Int3cArgs int3c_args(const Plan &p)
{
    Int3cArgs g{};
    g.pa = p.d.sp_a; g.pb = p.d.sp_b; g.pf0 = p.d.sp_f0; g.pq = p.d.sp_q;
    g.ao = ao_view(p); g.ax = ax_view(p);
    g.boys = p.d.boys; g.tau = p.thresh; g.ld = p.naux_pad;
    return g;
}

// Records of every kept pair into p.d.pair_rec (before any int3c launch).
void launch_pair_records(const Plan &p, hipStream_t s)
{
    int64_t off[7];
    pair_rec_offsets(p, off);
    Int3cArgs g = int3c_args(p);
    for (int pc = 0; pc < 6; ++pc) {
        g.p_begin = p.sp_class[pc].begin; g.p_end = p.sp_class[pc].end;
        double *rec = p.d.pair_rec + off[pc];
        switch (pc) {
        case 0: launch_pair_class<0, 0>(g, rec, s); break;
        case 1: launch_pair_class<1, 0>(g, rec, s); break;
        case 2: launch_pair_class<1, 1>(g, rec, s); break;
        case 3: launch_pair_class<2, 0>(g, rec, s); break;
        case 4: launch_pair_class<2, 1>(g, rec, s); break;
        default: launch_pair_class<2, 2>(g, rec, s); break;
        }
    }
}

template <int LA, int LB>
static void launch_pair_class_group(const Int3cArgs *args, double *const *recs, int n, hipStream_t s)
{
    constexpr int NAB = (2 * LA + 1) * (2 * LB + 1);
    PairRecGroup grp{};
    int64_t total = 0;
    auto flush = [&]() {
        if (grp.n == 0) return;
        grp.blk_start[grp.n] = (uint32_t)total;
        hipLaunchKernelGGL((k_pair_rec_group<LA, LB>), dim3((unsigned)total), dim3(256), 0, s, grp);
        grp = PairRecGroup{};
        total = 0;
    };
    for (int i = 0; i < n; ++i) {
        const int64_t nb = ((int64_t)(args[i].p_end - args[i].p_begin) * NAB + 255) / 256;
        if (nb <= 0) continue;
        if (grp.n == kPairRecGroupMax) flush();
        grp.blk_start[grp.n] = (uint32_t)total;
        grp.rec[grp.n] = recs[i];
        grp.g[grp.n++] = args[i];
        total += nb;
    }
    flush();
}

// Pair records of several plans, each class of all plans in shared launches.
void launch_pair_records_plans(const Plan *const *plans, int n, hipStream_t s)
{
    for (int pc = 0; pc < 6; ++pc) {
        std::vector<Int3cArgs> args;
        std::vector<double *> recs;
        for (int i = 0; i < n; ++i) {
            const Plan &p = *plans[i];
            int64_t off[7];
            pair_rec_offsets(p, off);
            Int3cArgs g = int3c_args(p);
            g.p_begin = p.sp_class[pc].begin; g.p_end = p.sp_class[pc].end;
            if (g.p_end <= g.p_begin) continue;
            args.push_back(g);
            recs.push_back(p.d.pair_rec + off[pc]);
        }
        const int m = (int)args.size();
        if (m == 0) continue;
        switch (pc) {
        case 0: launch_pair_class_group<0, 0>(args.data(), recs.data(), m, s); break;
        case 1: launch_pair_class_group<1, 0>(args.data(), recs.data(), m, s); break;
        case 2: launch_pair_class_group<1, 1>(args.data(), recs.data(), m, s); break;
        case 3: launch_pair_class_group<2, 0>(args.data(), recs.data(), m, s); break;
        case 4: launch_pair_class_group<2, 1>(args.data(), recs.data(), m, s); break;
        default: launch_pair_class_group<2, 2>(args.data(), recs.data(), m, s); break;
        }
    }
}

void launch_int3c(const Plan &p, hipStream_t s)
{
    launch_int3c_rows(p, p.d.U, 0, 0, (int32_t)p.sp_a.size(), s);
}

// U rows of the kept pairs i0 <= i < i1, written at row f - f_base of U
// (their pair records already formed by launch_pair_records).
void launch_int3c_rows(const Plan &p, double *U, int64_t f_base, int32_t i0, int32_t i1, hipStream_t s)
{
    int64_t off[7];
    pair_rec_offsets(p, off);
    Int3cArgs g = int3c_args(p);
    g.U = U; g.f_base = f_base;
    for (int pc = 0; pc < 6; ++pc) {
        g.p_begin = std::max(p.sp_class[pc].begin, i0); g.p_end = std::min(p.sp_class[pc].end, i1);
        if (g.p_end <= g.p_begin) continue;
        g.rec = p.d.pair_rec + off[pc];
        g.rec_first = p.sp_class[pc].begin;
        for (int lc = 0; lc <= kMaxLAux; ++lc) {
            g.c_begin = p.ax_class[lc].begin; g.c_end = p.ax_class[lc].end;
            if (g.c_end <= g.c_begin) continue;
            const int key = kPairClassLa[pc] * 100 + kPairClassLb[pc] * 10 + lc;
#define CLS(A, B, C) case A * 100 + B * 10 + C: launch_class<A, B, C>(g, s); break;
            switch (key) {
                CLS(0, 0, 0) CLS(0, 0, 1) CLS(0, 0, 2) CLS(0, 0, 3)
                CLS(1, 0, 0) CLS(1, 0, 1) CLS(1, 0, 2) CLS(1, 0, 3)
                CLS(1, 1, 0) CLS(1, 1, 1) CLS(1, 1, 2) CLS(1, 1, 3)
                CLS(2, 0, 0) CLS(2, 0, 1) CLS(2, 0, 2) CLS(2, 0, 3)
                CLS(2, 1, 0) CLS(2, 1, 1) CLS(2, 1, 2) CLS(2, 1, 3)
                CLS(2, 2, 0) CLS(2, 2, 1) CLS(2, 2, 2) CLS(2, 2, 3)
            }
#undef CLS
        }
    }
}

// The three-centre integrals of several set-up-in-progress plans (their
// pair records formed), every class's triplets of all plans in shared
// launches (up to kInt3cGroupMax plans each).
void launch_int3c_plans(const Plan *const *plans, int n, hipStream_t s)
{
    std::vector<Int3cArgs> args(n);
    std::vector<std::array<int64_t, 7>> off(n);
    for (int i = 0; i < n; ++i) {
        pair_rec_offsets(*plans[i], off[i].data());
        args[i] = int3c_args(*plans[i]);
        args[i].U = plans[i]->d.U;
        args[i].f_base = 0;
    }
    for (int pc = 0; pc < 6; ++pc)
        for (int lc = 0; lc <= kMaxLAux; ++lc) {
            std::vector<Int3cArgs> cls;
            for (int i = 0; i < n; ++i) {
                const Plan &p = *plans[i];
                Int3cArgs g = args[i];
                g.p_begin = p.sp_class[pc].begin; g.p_end = p.sp_class[pc].end;
                g.c_begin = p.ax_class[lc].begin; g.c_end = p.ax_class[lc].end;
                if (g.p_end <= g.p_begin || g.c_end <= g.c_begin) continue;
                g.rec = p.d.pair_rec + off[i][pc];
                g.rec_first = p.sp_class[pc].begin;
                cls.push_back(g);
            }
            if (cls.empty()) continue;
            const int key = kPairClassLa[pc] * 100 + kPairClassLb[pc] * 10 + lc;
            const int m = (int)cls.size();
#define CLS(A, B, C) case A * 100 + B * 10 + C: launch_class_group<A, B, C>(cls.data(), m, s); break;
            switch (key) {
                CLS(0, 0, 0) CLS(0, 0, 1) CLS(0, 0, 2) CLS(0, 0, 3)
                CLS(1, 0, 0) CLS(1, 0, 1) CLS(1, 0, 2) CLS(1, 0, 3)
                CLS(1, 1, 0) CLS(1, 1, 1) CLS(1, 1, 2) CLS(1, 1, 3)
                CLS(2, 0, 0) CLS(2, 0, 1) CLS(2, 0, 2) CLS(2, 0, 3)
                CLS(2, 1, 0) CLS(2, 1, 1) CLS(2, 1, 2) CLS(2, 1, 3)
                CLS(2, 2, 0) CLS(2, 2, 1) CLS(2, 2, 2) CLS(2, 2, 3)
            }
#undef CLS
        }
}

// --------------------------------------------------------------------------
// Pair tables of the four-centre direct path.  For pair i of class (LA, LB)
// (shells a, b): p = a + b, P = (aA + bB)/p and, for every function pair
// f = (ma, mb), the spherical Hermite expansion
//   E_f[tuv] = N_a N_b sum_{ca,cb} s_a[ma][ca] s_b[mb][cb] E^x E^y E^z,
// so that (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q))
//                   sum_{tuv} E_f[tuv] sum_{t'u'v'} (-1)^{t'+u'+v'} E_g[t'u'v'] R_{t+t',u+u',v+v'}.

template <int LA, int LB>
__global__ __launch_bounds__(128) void k_direct_pairs(DirectClassDev c, ShellsDev ao, double *px, double *py,
                                                      double *pz, double *pp, double *Eb, double *Ek)
{
    constexpr int NA = 2 * LA + 1, NB = 2 * LB + 1, NF = NA * NB, LAB = LA + LB, NH = nherm(LAB);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    const int a = c.sh_a[i], b = c.sh_b[i];
    const double ea = ao.exp[a], eb = ao.exp[b];
    const double Ax = ao.x[a], Ay = ao.y[a], Az = ao.z[a], Bx = ao.x[b], By = ao.y[b], Bz = ao.z[b];
    const double p = ea + eb, ip = 1.0 / p;
    const double Px = (ea * Ax + eb * Bx) * ip, Py = (ea * Ay + eb * By) * ip, Pz = (ea * Az + eb * Bz) * ip;
    const double mu = ea * eb * ip;
    double Ex[LA + 1][LB + 1][LAB + 1], Ey[LA + 1][LB + 1][LAB + 1], Ez[LA + 1][LB + 1][LAB + 1];
    hermite_E<LA, LB>(Px - Ax, Px - Bx, 0.5 * ip, exp(-mu * (Ax - Bx) * (Ax - Bx)), Ex);
    hermite_E<LA, LB>(Py - Ay, Py - By, 0.5 * ip, exp(-mu * (Ay - By) * (Ay - By)), Ey);
    hermite_E<LA, LB>(Pz - Az, Pz - Bz, 0.5 * ip, exp(-mu * (Az - Bz) * (Az - Bz)), Ez);
    px[i] = Px; py[i] = Py; pz[i] = Pz; pp[i] = p;
    const double nn = ao.norm[a] * ao.norm[b];
    for (int ma = 0; ma < NA; ++ma)
        for (int mb = 0; mb < NB; ++mb) {
            const int f = ma * NB + mb;
            double Es[NH];
            bra_sph<LA, LB>(ma, mb, Ex, Ey, Ez, Es);
#pragma unroll
            for (int t = 0; t <= LAB; ++t)
#pragma unroll
                for (int u = 0; u + t <= LAB; ++u)
#pragma unroll
                    for (int v = 0; v + u + t <= LAB; ++v) {
                        const int h = hidx(t, u, v);
                        const double e = nn * Es[h];
                        Eb[(int64_t)(f * NH + h) * c.npad + i] = e;
                        Ek[((int64_t)i * NF + f) * NH + h] = ((t + u + v) & 1) ? -e : e;
                    }
        }
}

void launch_direct_pairs(const DirectClassDev *cls, const ShellsDev &ao, hipStream_t s)
{
    for (int k = 0; k < 6; ++k) {
        const DirectClassDev &c = cls[k];
        if (c.n <= 0) continue;
        const dim3 grid((unsigned)((c.n + 127) / 128));
        double *px = const_cast<double *>(c.px), *py = const_cast<double *>(c.py), *pz = const_cast<double *>(c.pz);
        double *pp = const_cast<double *>(c.p), *Eb = const_cast<double *>(c.Eb), *Ek = const_cast<double *>(c.Ek);
        switch (k) {
        case 0: hipLaunchKernelGGL((k_direct_pairs<0, 0>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        case 1: hipLaunchKernelGGL((k_direct_pairs<1, 0>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        case 2: hipLaunchKernelGGL((k_direct_pairs<1, 1>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        case 3: hipLaunchKernelGGL((k_direct_pairs<2, 0>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        case 4: hipLaunchKernelGGL((k_direct_pairs<2, 1>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        default: hipLaunchKernelGGL((k_direct_pairs<2, 2>), grid, dim3(128), 0, s, c, ao, px, py, pz, pp, Eb, Ek); break;
        }
    }
}

// --------------------------------------------------------------------------
// Two-centre metric (P|Q), both sides solid harmonic (Hobson on each):
// (c|d) = N_c N_d 2 pi^{5/2}/(g d sqrt(g+d)) (2g)^{-lc} (-1)^{ld} (2d)^{-ld}
//         sum_{k,k'} s_c(k) s_d(k') R_{k+k'}(alpha, C-D).
// The sum over k' is S_md(grad) applied to R_000, which by Hobson's theorem is
// d^k [S_md(X, Y, Z) (-2 alpha)^ld F_ld(alpha r^2)]; with the Taylor-scaled
// tables of the three-centre kernel (G' to order lc, D of S_md) it is
// k! W'[k], W'[k] = sum_d D[d] G'[k - d], needed only at |k| = lc.  So
// (c|d) = N_c N_d 2 pi^{5/2}/(g d sqrt(g+d)) (2g)^{-lc} (g/(g+d))^ld
//         sum_{|k| = lc} s_c(k) k! W'[k].

struct Int2cArgs {
    ShellsDev ax;
    const double *boys;
    double *V;
    int64_t ld;
    int32_t nsh;
};

template <int LC, int LD>
__device__ void metric_block(const Int2cArgs &g, int c, int d)
{
    constexpr int CC = ncart(LC), CD = ncart(LD);
    const double gc = g.ax.exp[c], gd = g.ax.exp[d];
    const double X = g.ax.x[c] - g.ax.x[d], Y = g.ax.y[c] - g.ax.y[d], Z = g.ax.z[c] - g.ax.z[d];
    double G[nherm(LC)], M[nherm(LD)], sc;
    // ket_table with (p, g) = (gc, gd) gives G' = d^k F_ld(alpha r^2)/k! to order lc,
    // the monomials to order ld, and (alpha/gd)^ld / (gd sqrt(gc+gd)), alpha/gd = gc/(gc+gd)
    ket_table<LC, LD>(gc, X, Y, Z, gd, g.boys, G, M, sc);
#pragma unroll
    for (int k = 0; k < LC; ++k) sc *= 0.5 / gc;
    const double pref = kTwoPi52 / gc * sc * g.ax.norm[c] * g.ax.norm[d];
    const int oc = g.ax.off[c], od = g.ax.off[d];
#pragma unroll
    for (int md = 0; md < 2 * LD + 1; ++md) {
        double sv[CD], D[nherm(LD)];
#pragma unroll
        for (int k = 0; k < CD; ++k) sv[k] = c_sph[LD][md][k];
        ket_factor<LD>(sv, M, D);
        double W[CC];
#pragma unroll
        for (int i = 0; i < CC; ++i) {
            const int t = cart_pow(LC, i, 0), u = cart_pow(LC, i, 1), v = cart_pow(LC, i, 2);
            double w = 0.0;
#pragma unroll
            for (int dx = 0; dx <= t && dx <= LD; ++dx)
#pragma unroll
                for (int dy = 0; dy <= u && dx + dy <= LD; ++dy)
#pragma unroll
                    for (int dz = 0; dz <= v && dx + dy + dz <= LD; ++dz)
                        w += D[hidx(dx, dy, dz)] * G[hidx(t - dx, u - dy, v - dz)];
            W[i] = w * (kFact[t] * kFact[u] * kFact[v]);
        }
#pragma unroll
        for (int mc = 0; mc < 2 * LC + 1; ++mc) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < CC; ++i) s += c_sph[LC][mc][i] * W[i];
            s *= pref;
            g.V[(int64_t)(oc + mc) * g.ld + od + md] = s;
            g.V[(int64_t)(od + md) * g.ld + oc + mc] = s;
        }
    }
}

__global__ __launch_bounds__(128) void k_int2c(Int2cArgs g)
{
    const int64_t cd = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)g.nsh * (g.nsh + 1) / 2;
    if (cd >= n) return;
    int c = (int)((sqrt(8.0 * (double)cd + 1.0) - 1.0) * 0.5);
    while ((int64_t)c * (c + 1) / 2 > cd) --c;
    while ((int64_t)(c + 1) * (c + 2) / 2 <= cd) ++c;
    const int d = (int)(cd - (int64_t)c * (c + 1) / 2);
    const int key = g.ax.l[c] * 4 + g.ax.l[d];
#define MB(A, B) case A * 4 + B: metric_block<A, B>(g, c, d); break;
    switch (key) {
        MB(0, 0) MB(0, 1) MB(0, 2) MB(0, 3) MB(1, 0) MB(1, 1) MB(1, 2) MB(1, 3)
        MB(2, 0) MB(2, 1) MB(2, 2) MB(2, 3) MB(3, 0) MB(3, 1) MB(3, 2) MB(3, 3)
    }
#undef MB
}

void launch_int2c(const Plan &p, hipStream_t s)
{
    Int2cArgs g{ax_view(p), p.d.boys, p.d.V, p.naux_pad, p.nsh_aux};
    const int64_t n = (int64_t)p.nsh_aux * (p.nsh_aux + 1) / 2;
    const int bs = 128;
    hipLaunchKernelGGL(k_int2c, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, g);
}

}  // namespace dfjk
