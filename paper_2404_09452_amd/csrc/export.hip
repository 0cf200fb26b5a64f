// Diagnostic copies of the resident tensors in the caller's function order.
#include "dfjk_internal.h"

namespace dfjk {

__global__ void k_fill_export(double *p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

void launch_zero(double *p, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_export, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

__global__ void k_zero_rect(double *p, int64_t ld, int64_t r0, int64_t c0, int64_t nc, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[(r0 + i / nc) * ld + c0 + i % nc] = 0.0;
}

// zero rows r0..r1, columns c0..c1 of a row-major matrix with leading dimension ld
void launch_zero_rect(double *p, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t c1, hipStream_t s)
{
    const int64_t n = (r1 - r0) * (c1 - c0);
    if (r1 > r0 && c1 > c0)
        hipLaunchKernelGGL(k_zero_rect, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, ld, r0, c0, c1 - c0, n);
}

// out[Pc][mu][nu] = T[f][P] (and [Pc][nu][mu] for off-diagonal blocks)
__global__ void k_export_3c(const double *__restrict__ T, int64_t ld, const int32_t *__restrict__ fmu,
                            const int32_t *__restrict__ fnu, const double *__restrict__ fw,
                            const int32_t *__restrict__ fn_caller, int64_t nf, int64_t naux, int64_t nao,
                            double *__restrict__ out)
{
    const int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t f = blockIdx.y;
    if (P >= naux || f >= nf) return;
    const double v = T[f * ld + P];
    const int64_t Pc = fn_caller ? fn_caller[P] : P, mu = fmu[f], nu = fnu[f];
    out[(Pc * nao + mu) * nao + nu] = v;
    if (fw[f] > 1.5) out[(Pc * nao + nu) * nao + mu] = v;
}

__global__ void k_export_2c(const double *__restrict__ V, int64_t ld, const int32_t *__restrict__ fn_caller,
                            int64_t naux, int reorder, double *__restrict__ out)
{
    const int64_t Q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t P = blockIdx.y;
    if (Q >= naux || P >= naux) return;
    const int64_t Pc = reorder ? fn_caller[P] : P, Qc = reorder ? fn_caller[Q] : Q;
    out[Pc * naux + Qc] = V[P * ld + Q];
}

void launch_export(const Plan &p, int kind, double *out, hipStream_t s)
{
    if (kind == DFJK_EXPORT_INT3C || kind == DFJK_EXPORT_B) {
        const int64_t tot = p.naux * p.nao * p.nao;
        hipLaunchKernelGGL(k_fill_export, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, out, tot);
        if (p.nf == 0) return;
        const double *T = kind == DFJK_EXPORT_INT3C ? p.d.U : p.d.B;
        dim3 grid((unsigned)((p.naux + 255) / 256), (unsigned)p.nf);
        // B depends on the aux order through L, so it stays in the internal order
        const int32_t *order = kind == DFJK_EXPORT_INT3C ? p.d.ax_fn_caller : nullptr;
        hipLaunchKernelGGL(k_export_3c, grid, dim3(256), 0, s, T, p.naux_pad, p.d.f_mu, p.d.f_nu, p.d.f_w,
                           order, p.nf, p.naux, p.nao, out);
    } else {
        const double *M = kind == DFJK_EXPORT_METRIC ? p.d.V : p.d.L;
        dim3 grid((unsigned)((p.naux + 255) / 256), (unsigned)p.naux);
        hipLaunchKernelGGL(k_export_2c, grid, dim3(256), 0, s, M, p.naux_pad, p.d.ax_fn_caller, p.naux,
                           kind == DFJK_EXPORT_METRIC ? 1 : 0, out);
    }
}

// The dense pair map of the sampling diagnostic, built on the device from the
// stored rows: fmap[mu][nu] = f for the row f holding the pair (both
// orientations of an off-diagonal shell block), -1 elsewhere.
__global__ void k_fmap_clear(int32_t *__restrict__ fmap, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) fmap[i] = -1;
}

__global__ void k_fmap_rows(const int32_t *__restrict__ fmu, const int32_t *__restrict__ fnu,
                            const double *__restrict__ fw, int64_t nf, int64_t nao, int32_t *__restrict__ fmap)
{
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= nf) return;
    fmap[(int64_t)fmu[f] * nao + fnu[f]] = (int32_t)f;
    if (fw[f] > 1.5) fmap[(int64_t)fnu[f] * nao + fmu[f]] = (int32_t)f;
}

void launch_fmap(const Plan &p, hipStream_t s)
{
    const int64_t n = p.nao * p.nao;
    hipLaunchKernelGGL(k_fmap_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.d.fmap, n);
    if (p.nf > 0)
        hipLaunchKernelGGL(k_fmap_rows, dim3((unsigned)((p.nf + 255) / 256)), dim3(256), 0, s, p.d.f_mu, p.d.f_nu,
                           p.d.f_w, p.nf, p.nao, p.d.fmap);
}

// Sampled (P, mu, nu) -> value through the dense pair map fmap[mu][nu] = f or -1.
__global__ void k_sample(const double *__restrict__ T, int64_t ld, const int32_t *__restrict__ fmap,
                         const int32_t *__restrict__ fn_internal, int64_t naux, int64_t nao, int64_t n,
                         const int32_t *__restrict__ idx, double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t Pc = idx[3 * i], mu = idx[3 * i + 1], nu = idx[3 * i + 2];
    if (Pc < 0 || Pc >= naux || mu < 0 || mu >= nao || nu < 0 || nu >= nao) {
        out[i] = __builtin_nan("");   // index out of range
        return;
    }
    const int32_t f = fmap[(int64_t)mu * nao + nu];
    out[i] = (f < 0) ? 0.0 : T[(int64_t)f * ld + (fn_internal ? fn_internal[Pc] : Pc)];
}

void launch_sample(const Plan &p, int kind, int64_t n, const int32_t *idx, double *out, hipStream_t s)
{
    const double *T = kind == DFJK_EXPORT_INT3C ? p.d.U : p.d.B;
    const int32_t *to_internal = kind == DFJK_EXPORT_INT3C ? p.d.ax_fn_internal : nullptr;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, p.naux_pad, p.d.fmap,
                       to_internal, p.naux, p.nao, n, idx, out);
}

}  // namespace dfjk
