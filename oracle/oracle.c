/*
 * FP64 CPU oracle for the density-fitted Coulomb/exchange (DF-J/K) build.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the GPU
 * path is checked against.  It shares no code, header, table or generator
 * with the GPU library and must never be linked into it.
 *
 * The paper (GPU4PySCF v1.0, Introduction: density-fitted integrals followed
 * by tensor contractions) states none of the formulas; what is computed here
 * is the textbook definition, step by step:
 *   - Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt: a positive power
 *     series (long double) followed by the stable downward recursion for
 *     T <= 30, and erf plus upward recursion for T > 30.
 *   - Gaussian integrals by McMurchie-Davidson: Hermite expansion
 *     coefficients E^{ij}_t of each Cartesian product, Hermite Coulomb
 *     integrals R^n_{tuv} from the Boys function, then the Cartesian-to-
 *     spherical transform on every index.
 *   - Functions: phi = N_l(a) S_lm(r-A) exp(-a|r-A|^2), S_lm the real solid
 *     harmonics in Racah normalisation (p: x,y,z; d and f: m = -l..l),
 *     N_l chosen so that <phi|phi> = 1.
 *   - Plain column Cholesky of the metric and plain forward substitution.
 * Everything is unscreened.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LMAX 3             /* highest shell angular momentum handled       */
#define NCART_MAX 10       /* (LMAX+1)(LMAX+2)/2                            */
#define TMAX (4 * LMAX)    /* highest Hermite order, (ab|cd) at LMAX        */

/* ------------------------------------------------------------------------ */
/* Boys function                                                            */

void orc_boys(int mmax, double T, double *F)
{
    if (T <= 30.0) {
        /* F_M(T) = exp(-T) sum_k (2T)^k / ((2M+1)(2M+3)...(2M+2k+1)) */
        long double term = 1.0L / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 2000; k++) {
            term *= 2.0L * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-22L * sum) break;
        }
        long double e = expl(-(long double)T);
        long double f = e * sum;
        F[mmax] = (double)f;
        for (int m = mmax - 1; m >= 0; m--) {
            f = (2.0L * T * f + e) / (2 * m + 1);
            F[m] = (double)f;
        }
    } else {
        long double e = expl(-(long double)T);
        long double f = 0.5L * sqrtl(3.14159265358979323846264338327950288L / T) *
                        erfl(sqrtl((long double)T));
        F[0] = (double)f;
        for (int m = 0; m < mmax; m++) {
            f = ((2 * m + 1) * f - e) / (2.0L * T);
            F[m + 1] = (double)f;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Cartesian components and the spherical transform                          */

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian exponents in the order xx..., lx descending then ly descending */
static void cart_exponents(int l, int (*e)[3])
{
    int k = 0;
    for (int lx = l; lx >= 0; lx--)
        for (int ly = l - lx; ly >= 0; ly--) {
            e[k][0] = lx; e[k][1] = ly; e[k][2] = l - lx - ly; k++;
        }
}

static int cart_index(int l, int lx, int ly)
{
    /* position of (lx, ly, l-lx-ly) in cart_exponents order */
    int k = 0;
    for (int x = l; x > lx; x--) k += l - x + 1;
    return k + (l - lx - ly);
}

/* c[m][cart]: Racah-normalised real solid harmonics as monomial sums. */
static void sph_coeffs(int l, double c[7][NCART_MAX])
{
    memset(c, 0, sizeof(double) * 7 * NCART_MAX);
#define C(m, lx, ly, v) c[m][cart_index(l, lx, ly)] += (v)
    const double s3 = sqrt(3.0), s15 = sqrt(15.0), s58 = sqrt(5.0 / 8.0), s38 = sqrt(3.0 / 8.0);
    switch (l) {
    case 0: C(0, 0, 0, 1.0); break;
    case 1: C(0, 1, 0, 1.0); C(1, 0, 1, 1.0); C(2, 0, 0, 1.0); break;
    case 2:
        C(0, 1, 1, s3);                                   /* sqrt3 xy        */
        C(1, 0, 1, s3);                                   /* sqrt3 yz        */
        C(2, 0, 0, 1.0); C(2, 2, 0, -0.5); C(2, 0, 2, -0.5); /* z2-(x2+y2)/2 */
        C(3, 1, 0, s3);                                   /* sqrt3 xz        */
        C(4, 2, 0, 0.5 * s3); C(4, 0, 2, -0.5 * s3);      /* sqrt3/2 (x2-y2) */
        break;
    case 3:
        C(0, 2, 1, 3.0 * s58); C(0, 0, 3, -s58);          /* m=-3            */
        C(1, 1, 1, s15);                                  /* m=-2 xyz        */
        C(2, 0, 1, 4.0 * s38); C(2, 2, 1, -s38); C(2, 0, 3, -s38); /* m=-1 */
        C(3, 0, 0, 1.0); C(3, 2, 0, -1.5); C(3, 0, 2, -1.5);        /* m=0  */
        C(4, 1, 0, 4.0 * s38); C(4, 3, 0, -s38); C(4, 1, 2, -s38); /* m=1  */
        C(5, 2, 0, 0.5 * s15); C(5, 0, 2, -0.5 * s15);    /* m=2             */
        C(6, 3, 0, s58); C(6, 1, 2, -3.0 * s58);          /* m=3             */
        break;
    }
#undef C
}

static double dfact(int n) /* n!! with (-1)!! = 1 */
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

/* N_l(a): <phi|phi> = 1 for phi = N S_lm(r) exp(-a r^2), every m. */
double orc_norm(int l, double a)
{
    const double pi = 3.14159265358979323846;
    double radial = dfact(2 * l + 1) / (pow(2.0, l + 2) * pow(2.0 * a, l + 1)) *
                    sqrt(pi / (2.0 * a));
    double angular = 4.0 * pi / (2 * l + 1);
    return 1.0 / sqrt(radial * angular);
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson building blocks                                        */

/* E[i][j][t], i <= la, j <= lb, for the 1-D product of exponents a (at A)
 * and b (at B).  b == 0 gives the expansion of a single Gaussian at A. */
typedef double Etab[LMAX + 1][LMAX + 1][2 * LMAX + 1];

static void hermite_E(int la, int lb, double a, double b, double A, double B, Etab E)
{
    memset(E, 0, sizeof(Etab));
    double p = a + b, mu = a * b / p, X = A - B;
    double P = (a * A + b * B) / p, XPA = P - A, XPB = P - B, h = 0.5 / p;
    E[0][0][0] = exp(-mu * X * X);
    for (int i = 0; i < la; i++)
        for (int t = 0; t <= i + 1; t++) {
            double v = XPA * E[i][0][t];
            if (t > 0) v += h * E[i][0][t - 1];
            if (t + 1 <= i) v += (t + 1) * E[i][0][t + 1];
            E[i + 1][0][t] = v;
        }
    for (int i = 0; i <= la; i++)
        for (int j = 0; j < lb; j++)
            for (int t = 0; t <= i + j + 1; t++) {
                double v = XPB * E[i][j][t];
                if (t > 0) v += h * E[i][j][t - 1];
                if (t + 1 <= i + j) v += (t + 1) * E[i][j][t + 1];
                E[i][j + 1][t] = v;
            }
}

/* Hermite Coulomb integrals R^0_{tuv}(alpha, PC) for t+u+v <= L, stored in
 * R[(t*(L+1) + u)*(L+1) + v].  work must hold (L+1)^4 doubles. */
static void hermite_R(int L, double alpha, double X, double Y, double Z, double *R, double *work)
{
    int n1 = L + 1;
#define IDX(n, t, u, v) ((((n) * n1 + (t)) * n1 + (u)) * n1 + (v))
    double F[TMAX + 1];
    orc_boys(L, alpha * (X * X + Y * Y + Z * Z), F);
    double m2a = -2.0 * alpha, pw = 1.0;
    for (int n = 0; n <= L; n++) { work[IDX(n, 0, 0, 0)] = pw * F[n]; pw *= m2a; }
    for (int n = L - 1; n >= 0; n--)
        for (int t = 0; t <= L - n; t++)
            for (int u = 0; u <= L - n - t; u++)
                for (int v = 0; v <= L - n - t - u; v++) {
                    if (t + u + v == 0) continue;
                    double r;
                    if (t > 0) {
                        r = X * work[IDX(n + 1, t - 1, u, v)];
                        if (t > 1) r += (t - 1) * work[IDX(n + 1, t - 2, u, v)];
                    } else if (u > 0) {
                        r = Y * work[IDX(n + 1, t, u - 1, v)];
                        if (u > 1) r += (u - 1) * work[IDX(n + 1, t, u - 2, v)];
                    } else {
                        r = Z * work[IDX(n + 1, t, u, v - 1)];
                        if (v > 1) r += (v - 1) * work[IDX(n + 1, t, u, v - 2)];
                    }
                    work[IDX(n, t, u, v)] = r;
                }
    for (int t = 0; t <= L; t++)
        for (int u = 0; u <= L - t; u++)
            for (int v = 0; v <= L - t - u; v++)
                R[(t * n1 + u) * n1 + v] = work[IDX(0, t, u, v)];
#undef IDX
}

/* A charge distribution: the product of two shells (or one shell, b = 0),
 * expanded in Hermite Gaussians at its centre P with exponent p. */
typedef struct {
    int la, lb, na, nb;          /* Cartesian counts                      */
    double p, P[3];
    Etab E[3];                   /* per direction                          */
    int ea[NCART_MAX][3], eb[NCART_MAX][3];
} Dist;

static void make_dist(Dist *d, int la, double a, const double *A, int lb, double b, const double *B)
{
    d->la = la; d->lb = lb; d->na = ncart(la); d->nb = ncart(lb);
    d->p = a + b;
    for (int x = 0; x < 3; x++) {
        d->P[x] = (a * A[x] + b * B[x]) / d->p;
        hermite_E(la, lb, a, b, A[x], B[x], d->E[x]);
    }
    cart_exponents(la, d->ea);
    cart_exponents(lb, d->eb);
}

/* Cartesian Coulomb integrals between two distributions:
 * out[(ia*nb1 + ib)*(nc*nd) + ic*nd + id]. */
static void coulomb_cart(const Dist *d1, const Dist *d2, double *out, double *Rbuf, double *work)
{
    const double pi = 3.14159265358979323846;
    int L = d1->la + d1->lb + d2->la + d2->lb, n1 = L + 1;
    double p = d1->p, q = d2->p, alpha = p * q / (p + q);
    double pref = 2.0 * pow(pi, 2.5) / (p * q * sqrt(p + q));
    hermite_R(L, alpha, d1->P[0] - d2->P[0], d1->P[1] - d2->P[1], d1->P[2] - d2->P[2], Rbuf, work);
    int n2 = d2->na * d2->nb;
    for (int ia = 0; ia < d1->na; ia++)
        for (int ib = 0; ib < d1->nb; ib++) {
            const int *xa = d1->ea[ia], *xb = d1->eb[ib];
            for (int ic = 0; ic < d2->na; ic++)
                for (int id = 0; id < d2->nb; id++) {
                    const int *xc = d2->ea[ic], *xd = d2->eb[id];
                    double s = 0.0;
                    for (int t = 0; t <= xa[0] + xb[0]; t++)
                        for (int u = 0; u <= xa[1] + xb[1]; u++)
                            for (int v = 0; v <= xa[2] + xb[2]; v++) {
                                double e1 = d1->E[0][xa[0]][xb[0]][t] * d1->E[1][xa[1]][xb[1]][u] *
                                            d1->E[2][xa[2]][xb[2]][v];
                                if (e1 == 0.0) continue;
                                double inner = 0.0;
                                for (int tt = 0; tt <= xc[0] + xd[0]; tt++)
                                    for (int uu = 0; uu <= xc[1] + xd[1]; uu++)
                                        for (int vv = 0; vv <= xc[2] + xd[2]; vv++) {
                                            double e2 = d2->E[0][xc[0]][xd[0]][tt] *
                                                        d2->E[1][xc[1]][xd[1]][uu] *
                                                        d2->E[2][xc[2]][xd[2]][vv];
                                            double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                                            inner += sg * e2 * Rbuf[((t + tt) * n1 + (u + uu)) * n1 + (v + vv)];
                                        }
                                s += e1 * inner;
                            }
                    out[(ia * d1->nb + ib) * n2 + ic * d2->nb + id] = pref * s;
                }
        }
}

/* Apply the normalised spherical transform to index k (of 4) of a Cartesian
 * block with dims nc[4] (spherical dims ns[4]); in and out may not alias. */
static void sph_transform4(const double *in, double *out, const int *l, const double *expo)
{
    int nc[4], ns[4];
    double c[4][7][NCART_MAX];
    for (int k = 0; k < 4; k++) {
        nc[k] = ncart(l[k]); ns[k] = 2 * l[k] + 1;
        sph_coeffs(l[k], c[k]);
        double N = orc_norm(l[k], expo[k]);
        for (int m = 0; m < ns[k]; m++)
            for (int x = 0; x < nc[k]; x++) c[k][m][x] *= N;
    }
    for (int m0 = 0; m0 < ns[0]; m0++)
        for (int m1 = 0; m1 < ns[1]; m1++)
            for (int m2 = 0; m2 < ns[2]; m2++)
                for (int m3 = 0; m3 < ns[3]; m3++) {
                    double s = 0.0;
                    for (int x0 = 0; x0 < nc[0]; x0++) {
                        if (c[0][m0][x0] == 0.0) continue;
                        for (int x1 = 0; x1 < nc[1]; x1++) {
                            if (c[1][m1][x1] == 0.0) continue;
                            for (int x2 = 0; x2 < nc[2]; x2++) {
                                if (c[2][m2][x2] == 0.0) continue;
                                for (int x3 = 0; x3 < nc[3]; x3++) {
                                    if (c[3][m3][x3] == 0.0) continue;
                                    s += c[0][m0][x0] * c[1][m1][x1] * c[2][m2][x2] * c[3][m3][x3] *
                                         in[((x0 * nc[1] + x1) * nc[2] + x2) * nc[3] + x3];
                                }
                            }
                        }
                    }
                    out[((m0 * ns[1] + m1) * ns[2] + m2) * ns[3] + m3] = s;
                }
}

/* ------------------------------------------------------------------------ */
/* Public integral routines.  A basis is (nshell, atom[], l[], exp[]) with  */
/* function offsets in shell order, 2l+1 functions per shell.               */

static int *offsets(int n, const int *l)
{
    int *o = (int *)malloc(sizeof(int) * (n + 1));
    o[0] = 0;
    for (int i = 0; i < n; i++) o[i + 1] = o[i] + 2 * l[i] + 1;
    return o;
}

#define WORK_DOUBLES ((TMAX + 1) * (TMAX + 1) * (TMAX + 1) * (TMAX + 1))
#define RBUF_DOUBLES ((TMAX + 1) * (TMAX + 1) * (TMAX + 1))
#define BLK (NCART_MAX * NCART_MAX * NCART_MAX * NCART_MAX)

/* (mu nu | P) for every AO pair and the aux shells [c0, c1):
 * out[(P - P0) * nao * nao + mu * nao + nu], both AO triangles filled. */
int orc_int3c(const double *coords,
              int nao_sh, const int *ao_atom, const int *ao_l, const double *ao_exp,
              int nax_sh, const int *ax_atom, const int *ax_l, const double *ax_exp,
              int c0, int c1, double *out)
{
    for (int i = 0; i < nao_sh; i++) if (ao_l[i] < 0 || ao_l[i] > LMAX) return 1;
    for (int i = 0; i < nax_sh; i++) if (ax_l[i] < 0 || ax_l[i] > LMAX) return 1;
    int *ao = offsets(nao_sh, ao_l), *ax = offsets(nax_sh, ax_l);
    int nao = ao[nao_sh];
    long P0 = ax[c0];
    long npair = (long)nao_sh * (nao_sh + 1) / 2;
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * WORK_DOUBLES);
        double *Rb = (double *)malloc(sizeof(double) * RBUF_DOUBLES);
        double *cart = (double *)malloc(sizeof(double) * BLK);
        double *sph = (double *)malloc(sizeof(double) * BLK);
#pragma omp for schedule(dynamic, 4)
        for (long ab = 0; ab < npair; ab++) {
            int a = (int)((sqrt(8.0 * ab + 1.0) - 1.0) / 2.0);
            while ((long)a * (a + 1) / 2 > ab) a--;
            while ((long)(a + 1) * (a + 2) / 2 <= ab) a++;
            int b = (int)(ab - (long)a * (a + 1) / 2);
            Dist d1;
            make_dist(&d1, ao_l[a], ao_exp[a], coords + 3 * ao_atom[a], ao_l[b], ao_exp[b],
                      coords + 3 * ao_atom[b]);
            for (int c = c0; c < c1; c++) {
                Dist d2;
                const double *C = coords + 3 * ax_atom[c];
                make_dist(&d2, ax_l[c], ax_exp[c], C, 0, 0.0, C);
                coulomb_cart(&d1, &d2, cart, Rb, work);
                int ls[4] = {ao_l[a], ao_l[b], ax_l[c], 0};
                double ex[4] = {ao_exp[a], ao_exp[b], ax_exp[c], 1.0};
                sph_transform4(cart, sph, ls, ex);
                /* the l=0 dummy index got N_0(1); undo it */
                double n0 = orc_norm(0, 1.0);
                int na = 2 * ao_l[a] + 1, nb = 2 * ao_l[b] + 1, nc = 2 * ax_l[c] + 1;
                for (int i = 0; i < na; i++)
                    for (int j = 0; j < nb; j++)
                        for (int k = 0; k < nc; k++) {
                            double v = sph[(i * nb + j) * nc + k] / n0;
                            long P = ax[c] + k - P0;
                            out[P * nao * nao + (long)(ao[a] + i) * nao + ao[b] + j] = v;
                            out[P * nao * nao + (long)(ao[b] + j) * nao + ao[a] + i] = v;
                        }
            }
        }
        free(work); free(Rb); free(cart); free(sph);
    }
    free(ao); free(ax);
    return 0;
}

/* Two-centre Coulomb metric (P|Q), full naux x naux. */
int orc_int2c(const double *coords, int nsh, const int *atom, const int *l, const double *expo,
              double *out)
{
    for (int i = 0; i < nsh; i++) if (l[i] < 0 || l[i] > LMAX) return 1;
    int *o = offsets(nsh, l);
    int n = o[nsh];
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * WORK_DOUBLES);
        double *Rb = (double *)malloc(sizeof(double) * RBUF_DOUBLES);
        double *cart = (double *)malloc(sizeof(double) * BLK);
        double *sph = (double *)malloc(sizeof(double) * BLK);
#pragma omp for schedule(dynamic, 4)
        for (int c = 0; c < nsh; c++)
            for (int d = 0; d <= c; d++) {
                Dist d1, d2;
                const double *C = coords + 3 * atom[c], *D = coords + 3 * atom[d];
                make_dist(&d1, l[c], expo[c], C, 0, 0.0, C);
                make_dist(&d2, l[d], expo[d], D, 0, 0.0, D);
                coulomb_cart(&d1, &d2, cart, Rb, work);
                int ls[4] = {l[c], 0, l[d], 0};
                double ex[4] = {expo[c], 1.0, expo[d], 1.0};
                sph_transform4(cart, sph, ls, ex);
                double n0 = orc_norm(0, 1.0);
                int nc = 2 * l[c] + 1, nd = 2 * l[d] + 1;
                for (int i = 0; i < nc; i++)
                    for (int k = 0; k < nd; k++) {
                        double v = sph[i * nd + k] / (n0 * n0);
                        out[(long)(o[c] + i) * n + o[d] + k] = v;
                        out[(long)(o[d] + k) * n + o[c] + i] = v;
                    }
            }
        free(work); free(Rb); free(cart); free(sph);
    }
    free(o);
    return 0;
}

/* Four-centre (mu nu | la si), full nao^4 (tiny systems only). */
int orc_int4c(const double *coords, int nsh, const int *atom, const int *l, const double *expo,
              double *out)
{
    for (int i = 0; i < nsh; i++) if (l[i] < 0 || l[i] > LMAX) return 1;
    int *o = offsets(nsh, l);
    long n = o[nsh];
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * WORK_DOUBLES);
        double *Rb = (double *)malloc(sizeof(double) * RBUF_DOUBLES);
        double *cart = (double *)malloc(sizeof(double) * BLK);
        double *sph = (double *)malloc(sizeof(double) * BLK);
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int a = 0; a < nsh; a++)
            for (int b = 0; b < nsh; b++) {
                Dist d1;
                make_dist(&d1, l[a], expo[a], coords + 3 * atom[a], l[b], expo[b], coords + 3 * atom[b]);
                for (int c = 0; c < nsh; c++)
                    for (int d = 0; d < nsh; d++) {
                        Dist d2;
                        make_dist(&d2, l[c], expo[c], coords + 3 * atom[c], l[d], expo[d],
                                  coords + 3 * atom[d]);
                        coulomb_cart(&d1, &d2, cart, Rb, work);
                        int ls[4] = {l[a], l[b], l[c], l[d]};
                        double ex[4] = {expo[a], expo[b], expo[c], expo[d]};
                        sph_transform4(cart, sph, ls, ex);
                        int na = 2 * l[a] + 1, nb = 2 * l[b] + 1, nc = 2 * l[c] + 1, nd = 2 * l[d] + 1;
                        for (int i = 0; i < na; i++)
                            for (int j = 0; j < nb; j++)
                                for (int k = 0; k < nc; k++)
                                    for (int m = 0; m < nd; m++)
                                        out[(((o[a] + i) * n + o[b] + j) * n + o[c] + k) * n + o[d] + m] =
                                            sph[((i * nb + j) * nc + k) * nd + m];
                    }
            }
        free(work); free(Rb); free(cart); free(sph);
    }
    free(o);
    return 0;
}

/* Exact (unfitted, unscreened) J and K blocks at chosen shell pairs, from the
 * definitions J_{mu nu} = sum_{la si} (mu nu|la si) D_{la si} and
 * K_{mu nu} = sum_{la si} (mu la|nu si) D_{la si} over every shell of the
 * basis.  D is nao x nao (row-major, used as given).  Request k asks for
 * the block of shells (ra[k], rc[k]); its (2l_a+1) x (2l_c+1) values go to
 * J and K at offset boff[k], row-major. */
int orc_jk_blocks(const double *coords, int nsh, const int *atom, const int *l, const double *expo,
                  const double *D, int nreq, const int *ra, const int *rc, const long *boff, double *J, double *K)
{
    for (int i = 0; i < nsh; i++) if (l[i] < 0 || l[i] > LMAX) return 1;
    for (int k = 0; k < nreq; k++) if (ra[k] < 0 || ra[k] >= nsh || rc[k] < 0 || rc[k] >= nsh) return 2;
    int *o = offsets(nsh, l);
    long n = o[nsh];
    for (int k = 0; k < nreq; k++) {
        const int a = ra[k], c = rc[k];
        const int na = 2 * l[a] + 1, nc = 2 * l[c] + 1;
        double *Jb = J + boff[k], *Kb = K + boff[k];
        for (int i = 0; i < na * nc; i++) { Jb[i] = 0.0; Kb[i] = 0.0; }
#pragma omp parallel
        {
            double *work = (double *)malloc(sizeof(double) * WORK_DOUBLES);
            double *Rb = (double *)malloc(sizeof(double) * RBUF_DOUBLES);
            double *cart = (double *)malloc(sizeof(double) * BLK);
            double *sph = (double *)malloc(sizeof(double) * BLK);
            double *jl = (double *)calloc((size_t)na * nc, sizeof(double));
            double *kl = (double *)calloc((size_t)na * nc, sizeof(double));
#pragma omp for schedule(dynamic, 1)
            for (int b = 0; b < nsh; b++) {
                const int nb = 2 * l[b] + 1;
                Dist dab, dac;
                make_dist(&dab, l[a], expo[a], coords + 3 * atom[a], l[b], expo[b], coords + 3 * atom[b]);
                make_dist(&dac, l[a], expo[a], coords + 3 * atom[a], l[c], expo[c], coords + 3 * atom[c]);
                for (int d = 0; d < nsh; d++) {
                    const int nd = 2 * l[d] + 1;
                    /* J: (a c | b d) D_bd */
                    Dist dbd;
                    make_dist(&dbd, l[b], expo[b], coords + 3 * atom[b], l[d], expo[d], coords + 3 * atom[d]);
                    coulomb_cart(&dac, &dbd, cart, Rb, work);
                    int lj[4] = {l[a], l[c], l[b], l[d]};
                    double ej[4] = {expo[a], expo[c], expo[b], expo[d]};
                    sph_transform4(cart, sph, lj, ej);
                    for (int i = 0; i < na; i++)
                        for (int j = 0; j < nc; j++)
                            for (int x = 0; x < nb; x++)
                                for (int y = 0; y < nd; y++)
                                    jl[i * nc + j] += sph[((i * nc + j) * nb + x) * nd + y] *
                                                      D[(o[b] + x) * n + o[d] + y];
                    /* K: (a b | c d) D_bd */
                    Dist dcd;
                    make_dist(&dcd, l[c], expo[c], coords + 3 * atom[c], l[d], expo[d], coords + 3 * atom[d]);
                    coulomb_cart(&dab, &dcd, cart, Rb, work);
                    int lk[4] = {l[a], l[b], l[c], l[d]};
                    double ek[4] = {expo[a], expo[b], expo[c], expo[d]};
                    sph_transform4(cart, sph, lk, ek);
                    for (int i = 0; i < na; i++)
                        for (int x = 0; x < nb; x++)
                            for (int j = 0; j < nc; j++)
                                for (int y = 0; y < nd; y++)
                                    kl[i * nc + j] += sph[((i * nb + x) * nc + j) * nd + y] *
                                                      D[(o[b] + x) * n + o[d] + y];
                }
            }
#pragma omp critical
            for (int i = 0; i < na * nc; i++) { Jb[i] += jl[i]; Kb[i] += kl[i]; }
            free(work); free(Rb); free(cart); free(sph); free(jl); free(kl);
        }
    }
    free(o);
    return 0;
}

/* Overlap S_{mu nu} = (pi/p)^{3/2} E^x_0 E^y_0 E^z_0, normalised, spherical. */
int orc_overlap(const double *coords, int nsh, const int *atom, const int *l, const double *expo,
                double *out)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < nsh; i++) if (l[i] < 0 || l[i] > LMAX) return 1;
    int *o = offsets(nsh, l);
    int n = o[nsh];
    for (int a = 0; a < nsh; a++)
        for (int b = 0; b <= a; b++) {
            Dist d;
            make_dist(&d, l[a], expo[a], coords + 3 * atom[a], l[b], expo[b], coords + 3 * atom[b]);
            double cart[NCART_MAX * NCART_MAX * NCART_MAX * NCART_MAX], sph[BLK];
            double pre = pow(pi / d.p, 1.5);
            for (int ia = 0; ia < d.na; ia++)
                for (int ib = 0; ib < d.nb; ib++) {
                    const int *xa = d.ea[ia], *xb = d.eb[ib];
                    cart[ia * d.nb + ib] = pre * d.E[0][xa[0]][xb[0]][0] * d.E[1][xa[1]][xb[1]][0] *
                                           d.E[2][xa[2]][xb[2]][0];
                }
            int ls[4] = {l[a], l[b], 0, 0};
            double ex[4] = {expo[a], expo[b], 1.0, 1.0};
            sph_transform4(cart, sph, ls, ex);
            double n0 = orc_norm(0, 1.0);
            int na = 2 * l[a] + 1, nb = 2 * l[b] + 1;
            for (int i = 0; i < na; i++)
                for (int j = 0; j < nb; j++) {
                    double v = sph[i * nb + j] / (n0 * n0);
                    out[(long)(o[a] + i) * n + o[b] + j] = v;
                    out[(long)(o[b] + j) * n + o[a] + i] = v;
                }
        }
    free(o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Linear algebra                                                            */

/* V = L L^T, plain column algorithm (L lower, row-major, upper part zero).
 * Returns -1 on success or the index of the first pivot <= 0. */
long orc_cholesky(long n, const double *V, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (long j = 0; j < n; j++) {
        double d = V[j * n + j];
        for (long k = 0; k < j; k++) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return j;
        double ljj = sqrt(d);
        L[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (long i = j + 1; i < n; i++) {
            double s = V[i * n + j];
            for (long k = 0; k < j; k++) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / ljj;
        }
    }
    return -1;
}

/* Solve L X = B in place for m right-hand sides: B is n x m row-major.
 * Row i of X is (B_i - sum_{k<i} L_ik X_k) / L_ii; columns are independent,
 * so threads take disjoint column ranges. */
void orc_forward_subst(long n, const double *L, long m, double *B)
{
    const long cw = 256;
    long nchunk = (m + cw - 1) / cw;
#pragma omp parallel for schedule(dynamic, 1)
    for (long ch = 0; ch < nchunk; ch++) {
        long c0 = ch * cw, c1 = c0 + cw < m ? c0 + cw : m;
        for (long i = 0; i < n; i++) {
            double *bi = B + i * m;
            for (long k = 0; k < i; k++) {
                double lik = L[i * n + k];
                const double *bk = B + k * m;
                for (long c = c0; c < c1; c++) bi[c] -= lik * bk[c];
            }
            double lii = L[i * n + i];
            for (long c = c0; c < c1; c++) bi[c] /= lii;
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
