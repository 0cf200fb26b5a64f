// Device building blocks for Gaussian integrals over solid-harmonic shells:
// the Boys function from a Taylor table, McMurchie-Davidson Hermite Coulomb
// integrals R_{tuv} and Hermite expansion coefficients E^{ij}_t.
// Everything is templated on the angular momenta so loops unroll and every
// table index is a compile-time constant.
#pragma once

#include <hip/hip_runtime.h>

#include "dfjk_internal.h"

namespace dfjk {

constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// number of Hermite indices (t,u,v) with t+u+v <= L
constexpr int nherm(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
// tetrahedral position of (t,u,v): grouped by order, then by u+v, then v
constexpr int hidx(int t, int u, int v)
{
    return (t + u + v) * (t + u + v + 1) * (t + u + v + 2) / 6 + (u + v) * (u + v + 1) / 2 + v;
}
// exponent `which` (0 x, 1 y, 2 z) of Cartesian component c of an l shell,
// components ordered lx descending, then ly descending
constexpr int cart_pow(int l, int c, int which)
{
    int k = 0;
    for (int lx = l; lx >= 0; --lx)
        for (int ly = l - lx; ly >= 0; --ly) {
            if (k == c) return which == 0 ? lx : (which == 1 ? ly : l - lx - ly);
            ++k;
        }
    return 0;
}
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi52 = 34.98683665524972;   // 2 pi^{5/2}

// F_0..F_M at T.  Below kBoysTMax: seven-term Taylor series of F_M about the
// nearest table point (dF_m/dT = -F_{m+1}), then downward recursion
// F_m = (2T F_{m+1} + e^{-T}) / (2m+1).  Above: F_0 = sqrt(pi/T)/2 (erf(sqrt T)
// is 1 to double precision there) and upward recursion
// F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T).
template <int M>
__device__ __forceinline__ void boys(double T, double (&F)[M + 1], const double *__restrict__ tab)
{
    if (T < kBoysTMax) {
        const int k = (int)(T * (1.0 / kBoysH) + 0.5);
        const double d = k * kBoysH - T;
        const double *row = tab + k * kBoysNM + M;
        double f = row[6];
        f = row[5] + d * (1.0 / 6.0) * f;
        f = row[4] + d * (1.0 / 5.0) * f;
        f = row[3] + d * (1.0 / 4.0) * f;
        f = row[2] + d * (1.0 / 3.0) * f;
        f = row[1] + d * (1.0 / 2.0) * f;
        f = row[0] + d * f;
        F[M] = f;
        if constexpr (M > 0) {
            const double e = exp(-T);
#pragma unroll
            for (int m = M - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) * (1.0 / (2 * m + 1));
        }
    } else {
        const double e = exp(-T);
        const double it2 = 0.5 / T;
        F[0] = 0.5 * sqrt(kPi / T);
#pragma unroll
        for (int m = 0; m < M; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * it2;
    }
}

// R_{tuv}(alpha, X, Y, Z) for t+u+v <= L, in place from the top level down:
// R^n_{000} = (-2 alpha)^n F_n, and R^n_{tuv} from R^{n+1} by
// R_{t+1,u,v} = t R_{t-1,u,v} + X R_{t,u,v} (same in u with Y, v with Z).
// Orders are overwritten from the highest down, so the lower orders still
// hold level n+1 when they are read.  With S > 0 the table starts from level
// S instead of 0 and is divided by (-2 alpha)^S: the derivatives of
// F_S(alpha r^2) rather than of F_0 (F holds at least S + L + 1 values).
template <int L, int S = 0, int NF>
__device__ __forceinline__ void hermite_R(double alpha, double X, double Y, double Z,
                                          const double (&F)[NF], double (&R)[nherm(L)])
{
    static_assert(NF >= S + L + 1, "Boys values missing");
    double H[L + 1];
    double pw = 1.0;
    const double m2a = -2.0 * alpha;
#pragma unroll
    for (int n = 0; n <= L; ++n) { H[n] = pw * F[S + n]; pw *= m2a; }
    R[0] = H[L];
#pragma unroll
    for (int n = L - 1; n >= 0; --n) {
#pragma unroll
        for (int k = L - n; k >= 1; --k) {
#pragma unroll
            for (int t = k; t >= 0; --t) {
#pragma unroll
                for (int u = k - t; u >= 0; --u) {
                    const int v = k - t - u;
                    double r;
                    if (t > 0) {
                        r = X * R[hidx(t - 1, u, v)];
                        if (t > 1) r += (t - 1) * R[hidx(t - 2, u, v)];
                    } else if (u > 0) {
                        r = Y * R[hidx(t, u - 1, v)];
                        if (u > 1) r += (u - 1) * R[hidx(t, u - 2, v)];
                    } else {
                        r = Z * R[hidx(t, u, v - 1)];
                        if (v > 1) r += (v - 1) * R[hidx(t, u, v - 2)];
                    }
                    R[hidx(t, u, v)] = r;
                }
            }
        }
        R[0] = H[n];
    }
}

// Hermite coefficients of one Cartesian direction of a Gaussian product:
// E[i][j][t], E^{00}_0 = e00, and
// E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1},
// E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}.
template <int LA, int LB>
__device__ __forceinline__ void hermite_E(double xpa, double xpb, double h /* 1/(2p) */, double e00,
                                          double (&E)[LA + 1][LB + 1][LA + LB + 1])
{
    E[0][0][0] = e00;
#pragma unroll
    for (int i = 0; i < LA; ++i)
#pragma unroll
        for (int t = 0; t <= i + 1; ++t) {
            double v = (t <= i) ? xpa * E[i][0][t] : 0.0;
            if (t > 0) v += h * E[i][0][t - 1];
            if (t + 1 <= i) v += (t + 1) * E[i][0][t + 1];
            E[i + 1][0][t] = v;
        }
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j < LB; ++j)
#pragma unroll
            for (int t = 0; t <= i + j + 1; ++t) {
                double v = (t <= i + j) ? xpb * E[i][j][t] : 0.0;
                if (t > 0) v += h * E[i][j][t - 1];
                if (t + 1 <= i + j) v += (t + 1) * E[i][j][t + 1];
                E[i][j + 1][t] = v;
            }
}

}  // namespace dfjk
