// k_stats.hip -- one-point statistics in FP64 (Section "Step 1": means and
// mean shear; the one-point moments and the pseudo-dissipation used by the
// assembly of the terms).  Every reduction has a fixed order, so results are
// bit-reproducible run to run.
#include "gke_internal.h"

namespace gke {

// Sum over a 256-thread block in a fixed order; result valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

// Block (j, part) sums 1/NSPLIT of plane j for the four fields and adds the
// four results to sums[f][j][part] (one owner per slot: fixed order).
template <typename TI>
__global__ __launch_bounds__(256) void k_plane_sums(const TI *__restrict__ u,
                                                    const TI *__restrict__ v,
                                                    const TI *__restrict__ w,
                                                    const TI *__restrict__ p, int npl, int ny,
                                                    double *__restrict__ sums)
{
    __shared__ double sh[8];
    const int j = blockIdx.x, part = blockIdx.y;
    const int len = (npl + NSPLIT - 1) / NSPLIT;
    const int i0 = part * len, i1 = min(npl, i0 + len);
    const size_t off = (size_t)j * npl;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        a[0] += (double)u[off + i];
        a[1] += (double)v[off + i];
        a[2] += (double)w[off + i];
        a[3] += (double)p[off + i];
    }
    for (int f = 0; f < 4; ++f) {
        const double r = block_sum(a[f], sh);
        if (threadIdx.x == 0) sums[((size_t)f * ny + j) * NSPLIT + part] += r;
    }
}

hipError_t launch_plane_sums(hipStream_t st, const Dims &d, int f32, const void *u,
                             const void *v, const void *w, const void *p, double *sums)
{
    const int npl = d.nx * d.nz;
    dim3 grid(d.ny, NSPLIT);
    if (f32)
        hipLaunchKernelGGL(k_plane_sums<float>, grid, dim3(256), 0, st,
                           (const float *)u, (const float *)v, (const float *)w,
                           (const float *)p, npl, d.ny, sums);
    else
        hipLaunchKernelGGL(k_plane_sums<double>, grid, dim3(256), 0, st,
                           (const double *)u, (const double *)v, (const double *)w,
                           (const double *)p, npl, d.ny, sums);
    return hipGetLastError();
}

// S(y) = dU/dy with the five-point weights
__device__ void shear_rows(int ny, const double *w5, const int *j0, double *prof)
{
    for (int j = threadIdx.x; j < ny; j += blockDim.x) {
        double s = 0.0;
        for (int a = 0; a < 5; ++a) s += w5[j * 5 + a] * prof[P_U * ny + j0[j] + a];
        prof[P_S * ny + j] = s;
    }
}

__global__ void k_means(int ny, const double *__restrict__ sums, double inv_count,
                        const double *__restrict__ w5, const int *__restrict__ j0,
                        double *__restrict__ prof)
{
    for (int i = threadIdx.x; i < 4 * ny; i += blockDim.x) {
        double a = 0.0;
        for (int part = 0; part < NSPLIT; ++part) a += sums[(size_t)i * NSPLIT + part];
        prof[i] = a * inv_count;
    }
    __syncthreads();
    shear_rows(ny, w5, j0, prof);
}

__global__ void k_shear(int ny, const double *__restrict__ w5, const int *__restrict__ j0,
                        double *__restrict__ prof)
{
    shear_rows(ny, w5, j0, prof);
}

hipError_t launch_means(hipStream_t st, const Dims &d, const Tables &t, const double *sums,
                        double count, double *prof)
{
    const double inv = 1.0 / (count * (double)d.nx * (double)d.nz);
    hipLaunchKernelGGL(k_means, dim3(1), dim3(256), 0, st, d.ny, sums, inv, t.w5, t.j0, prof);
    return hipGetLastError();
}

hipError_t launch_shear(hipStream_t st, const Dims &d, const Tables &t, double *prof)
{
    hipLaunchKernelGGL(k_shear, dim3(1), dim3(256), 0, st, d.ny, t.w5, t.j0, prof);
    return hipGetLastError();
}

// One block per plane: reduce the per-block partials of the moment kernels.
__global__ void k_profiles(int ny, int nzb, int nkx, const double *__restrict__ momp,
                           const double *__restrict__ momg, double inv_pts, double inv_count,
                           double nu, double *__restrict__ prof)
{
    const int j = blockIdx.x;
    if (threadIdx.x != 0) return;
    const double *mp = momp + (size_t)j * NMOMP * nzb;
    double s[NMOMP];
    for (int k = 0; k < NMOMP; ++k) {
        double a = 0.0;
        for (int b = 0; b < nzb; ++b) a += mp[k * nzb + b];
        s[k] = a * inv_pts;
    }
    double g = 0.0;
    const double *mg = momg + (size_t)j * 3 * nkx;
    for (int i = 0; i < 3 * nkx; ++i) g += mg[i];
    prof[P_Q * ny + j] = s[MP_Q];
    prof[P_UV * ny + j] = s[MP_UV];
    prof[P_PV * ny + j] = s[MP_PV];
    prof[P_TX * ny + j] = s[MP_QU];
    prof[P_TY * ny + j] = s[MP_QV];
    prof[P_TZ * ny + j] = s[MP_QW];
    prof[P_EPS * ny + j] = nu * (s[MP_GY] + g * inv_count);
}

hipError_t launch_profiles(hipStream_t st, const Dims &d, const double *momp,
                           const double *momg, double count, double *prof)
{
    const double inv_count = 1.0 / count;
    const double inv_pts = inv_count / ((double)d.nx * (double)d.nz);
    hipLaunchKernelGGL(k_profiles, dim3(d.ny), dim3(64), 0, st, d.ny, d.nzb, d.nkx, momp, momg,
                       inv_pts, inv_count, d.nu, prof);
    return hipGetLastError();
}

__global__ void k_t14(int ny, const double *__restrict__ prof, double *__restrict__ t14)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ny * ny) return;
    const int j1 = i / ny, j2 = i - j1 * ny;
    // -4 <eps*>, eps* the average of the two points
    t14[i] = -2.0 * (prof[P_EPS * ny + j1] + prof[P_EPS * ny + j2]);
}

hipError_t launch_t14(hipStream_t st, const Dims &d, const double *prof, double *t14)
{
    const int n = d.ny * d.ny;
    hipLaunchKernelGGL(k_t14, dim3((n + 255) / 256), dim3(256), 0, st, d.ny, prof, t14);
    return hipGetLastError();
}

}  // namespace gke
