// k_stats.hip -- one-point statistics in FP64 (Section "Step 1": means and
// mean shear; the one-point moments and the pseudo-dissipation used by the
// assembly of the terms).  Every reduction has a fixed order, so results are
// bit-reproducible run to run.
#include <algorithm>

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
    // four elements per field in flight per thread: unconditional loads at
    // clamped indices, the ones past the end add nothing
    constexpr int U = 4;
    for (int i = i0 + threadIdx.x; i < i1; i += U * blockDim.x) {
        TI x[U][4];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const size_t ik = off + min(i + k * (int)blockDim.x, i1 - 1);
            x[k][0] = u[ik];
            x[k][1] = v[ik];
            x[k][2] = w[ik];
            x[k][3] = p[ik];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool ok = i + k * (int)blockDim.x < i1;
#pragma unroll
            for (int f = 0; f < 4; ++f) a[f] += ok ? (double)x[k][f] : 0.0;
        }
    }
    for (int f = 0; f < 4; ++f) {
        const double r = block_sum(a[f], sh);
        if (threadIdx.x == 0) sums[((size_t)f * ny + j) * NSPLIT + part] += r;
    }
}

// The split path's first scan: the plane sums of k_plane_sums and, per
// plane, the sum of (D u~)^2 + (D v~)^2 + (D w~)^2 of the raw fields (D: the
// five-point wall-normal weights of the plane, nodes j0[j] .. j0[j] + 4), from
// which the means kernel forms the gradient energy of the fluctuations
// (Section "Step 2": the pseudo-dissipation; the split spectra cannot give its
// wall-normal part without losing digits to cancellation, and forming it in
// the second scan needs every plane's four neighbours there).
// Block (part, chunk): GY_JC planes of one 1/NSPLIT column range.  A thread
// loads the window nodes of its column point once (GY_JC + 4 planes of u v w,
// interior chunks, where node j0[j] = j - 2) and keeps them in registers; the
// chunks at the walls, whose windows are clamped, load each plane's five nodes.
// Sums in FP64, one fixed-order block reduction per value.
constexpr int GY_JC = 4;
template <typename TI>
__global__ __launch_bounds__(256) void k_plane_sums_gy(const TI *__restrict__ u,
                                                       const TI *__restrict__ v,
                                                       const TI *__restrict__ w,
                                                       const TI *__restrict__ p, int npl, int ny,
                                                       Tables t, double *__restrict__ sums)
{
    constexpr int NV = 5 * GY_JC, NV8 = (NV + 7) / 8 * 8;   // values, in groups of eight
    __shared__ double sh[NV8][4];
    __shared__ double sw[GY_JC][5];   // the planes' five-point weights
    const int part = blockIdx.x, ja = blockIdx.y * GY_JC;
    const int nj = min(GY_JC, ny - ja);
    const int len = (npl + NSPLIT - 1) / NSPLIT;
    const int i0 = part * len, i1 = min(npl, i0 + len);
    // interior: every plane's window starts two below it
    const bool interior = t.j0[ja] == ja - 2 && t.j0[ja + nj - 1] == ja + nj - 3;
    if ((int)threadIdx.x < 5 * GY_JC) {
        const int q = threadIdx.x / 5, k = threadIdx.x % 5;
        sw[q][k] = t.w5[(ja + min(q, nj - 1)) * 5 + k];
    }
    __syncthreads();
    double a[GY_JC][5];
#pragma unroll
    for (int q = 0; q < GY_JC; ++q)
#pragma unroll
        for (int f = 0; f < 5; ++f) a[q][f] = 0.0;
    for (int i = i0 + (int)threadIdx.x; i < i1; i += 256) {
        // an opaque zero added to the weight index keeps the weights in LDS,
        // read at each use: hoisted out of the loop they held 40 VGPRs (144 in
        // all, three waves per SIMD)
        int wz = 0;
        asm volatile("" : "+v"(wz));
        // plane bases are block-uniform (scalar registers); the lane offset is i
        TI pv[GY_JC];
#pragma unroll
        for (int q = 0; q < GY_JC; ++q) pv[q] = (p + (size_t)(ja + min(q, nj - 1)) * npl)[i];
        if (interior) {
            // nodes ja - 2 .. ja + nj + 1; slots past the chunk repeat its last node
            TI x[GY_JC + 4][3];
#pragma unroll
            for (int n = 0; n < GY_JC + 4; ++n) {
                const size_t o = (size_t)(ja - 2 + min(n, nj + 3)) * npl;
                x[n][0] = (u + o)[i];
                x[n][1] = (v + o)[i];
                x[n][2] = (w + o)[i];
            }
#pragma unroll
            for (int q = 0; q < GY_JC; ++q) {
                const bool ok = q < nj;
                const int j = ja + min(q, nj - 1);
                double du = 0.0, dv = 0.0, dw = 0.0;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const double wk = sw[q][k + wz];
                    du += wk * (double)x[q + k][0];
                    dv += wk * (double)x[q + k][1];
                    dw += wk * (double)x[q + k][2];
                }
                a[q][0] += ok ? (double)x[q + 2][0] : 0.0;
                a[q][1] += ok ? (double)x[q + 2][1] : 0.0;
                a[q][2] += ok ? (double)x[q + 2][2] : 0.0;
                a[q][3] += ok ? (double)pv[q] : 0.0;
                a[q][4] += ok ? du * du + dv * dv + dw * dw : 0.0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < GY_JC; ++q) {
                const bool ok = q < nj;
                const int j = ja + min(q, nj - 1), js = t.j0[j];
                TI x[5][3];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const size_t o = (size_t)(js + k) * npl;
                    x[k][0] = (u + o)[i];
                    x[k][1] = (v + o)[i];
                    x[k][2] = (w + o)[i];
                }
                const size_t oj = (size_t)j * npl;
                const double uj = (double)(u + oj)[i], vj = (double)(v + oj)[i];
                const double wj = (double)(w + oj)[i];
                double du = 0.0, dv = 0.0, dw = 0.0;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const double wk = sw[q][k + wz];
                    du += wk * (double)x[k][0];
                    dv += wk * (double)x[k][1];
                    dw += wk * (double)x[k][2];
                }
                a[q][0] += ok ? uj : 0.0;
                a[q][1] += ok ? vj : 0.0;
                a[q][2] += ok ? wj : 0.0;
                a[q][3] += ok ? (double)pv[q] : 0.0;
                a[q][4] += ok ? du * du + dv * dv + dw * dw : 0.0;
            }
        }
    }
    // NV values: wave reductions eight at a time (the last group padded with
    // zeros), then the four waves in order
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, g = lane >> 3;
#pragma unroll
    for (int c = 0; c < NV8 / 8; ++c) {
        double vals[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int vi = 8 * c + e;
            vals[e] = vi < NV ? a[vi / 5][vi % 5] : 0.0;
        }
        const double r = wave_sum8(vals);
        if ((lane & 7) == 0) sh[8 * c + g][wid] = r;
    }
    __syncthreads();
    if ((int)threadIdx.x < 5 * nj) {
        const int q = threadIdx.x / 5, f = threadIdx.x % 5;
        const double r = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] +
                         sh[threadIdx.x][3];
        sums[((size_t)f * ny + ja + q) * NSPLIT + part] += r;
    }
}

hipError_t launch_plane_sums(hipStream_t st, const Dims &d, const Tables &t, int f32, int gy,
                             const void *u, const void *v, const void *w, const void *p,
                             double *sums)
{
    const int npl = d.nx * d.nz;
    if (gy) {
        if (d.ny < 5) return hipErrorInvalidValue;
        dim3 grid(NSPLIT, (d.ny + GY_JC - 1) / GY_JC);
        if (f32)
            hipLaunchKernelGGL(k_plane_sums_gy<float>, grid, dim3(256), 0, st, (const float *)u,
                               (const float *)v, (const float *)w, (const float *)p, npl, d.ny,
                               t, sums);
        else
            hipLaunchKernelGGL(k_plane_sums_gy<double>, grid, dim3(256), 0, st, (const double *)u,
                               (const double *)v, (const double *)w, (const double *)p, npl,
                               d.ny, t, sums);
        return hipGetLastError();
    }
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
                        double *__restrict__ prof, double *__restrict__ gy1)
{
    for (int i = threadIdx.x; i < 4 * ny; i += blockDim.x) {
        double a = 0.0;
        for (int part = 0; part < NSPLIT; ++part) a += sums[(size_t)i * NSPLIT + part];
        prof[i] = a * inv_count;
    }
    __syncthreads();
    shear_rows(ny, w5, j0, prof);
    if (gy1) {
        // <(D u')^2> = <(D u~)^2> - (D U)^2 per component: D is linear and the
        // five-point D of the plane means is the plane mean of D u~
        for (int j = threadIdx.x; j < ny; j += blockDim.x) {
            double a = 0.0;
            for (int part = 0; part < NSPLIT; ++part)
                a += sums[((size_t)4 * ny + j) * NSPLIT + part];
            double dU = 0.0, dV = 0.0, dW = 0.0;
            for (int k = 0; k < 5; ++k) {
                const double wk = w5[j * 5 + k];
                const int n = j0[j] + k;
                dU += wk * prof[P_U * ny + n];
                dV += wk * prof[P_V * ny + n];
                dW += wk * prof[P_W * ny + n];
            }
            gy1[j] = a * inv_count - (dU * dU + dV * dV + dW * dW);
        }
    }
}

__global__ void k_shear(int ny, const double *__restrict__ w5, const int *__restrict__ j0,
                        double *__restrict__ prof)
{
    shear_rows(ny, w5, j0, prof);
}

hipError_t launch_means(hipStream_t st, const Dims &d, const Tables &t, const double *sums,
                        double count, double *prof, double *gy1)
{
    const double inv = 1.0 / (count * (double)d.nx * (double)d.nz);
    hipLaunchKernelGGL(k_means, dim3(1), dim3(256), 0, st, d.ny, sums, inv, t.w5, t.j0, prof,
                       gy1);
    return hipGetLastError();
}

hipError_t launch_shear(hipStream_t st, const Dims &d, const Tables &t, double *prof)
{
    hipLaunchKernelGGL(k_shear, dim3(1), dim3(256), 0, st, d.ny, t.w5, t.j0, prof);
    return hipGetLastError();
}

// One block per (plane Y, offset a = 0..4): the plane average of
// u'_i(Y) u'_i(Y + a), which by the Parseval identity over the stored half
// spectrum (weight 1 at kx = 0 and Nx/2, 2 otherwise) is
//   sum_k w_kx Re S_R(k; Y, Y + a) / count,
// and for a = 0 also the plane average of (d_x u'_i)^2 + (d_z u'_i)^2,
//   sum_k w_kx (alpha^2 + beta^2) S_R(k; Y, Y) / count
// (spectral derivatives, zero multiplier at the Nyquist wavenumbers).  These
// give the pseudo-dissipation (Section "Step 2") without further passes over
// the fields.  r0[Y][a], gxz[Y]; a fixed summation order.
__global__ __launch_bounds__(256) void k_r0(const cx<double> *__restrict__ acc, Dims d,
                                            Tables t, double inv_count, double *__restrict__ r0,
                                            double *__restrict__ gxz)
{
    __shared__ double sh[8];
    const int y = blockIdx.x, a = blockIdx.y;
    if (y + a >= d.ny) {
        if (threadIdx.x == 0) r0[y * 5 + a] = 0.0;
        return;
    }
    const int P = t.pidx[y * d.ny + y + a];
    const cx<double> *s = acc + (size_t)S_R * d.nk * d.pstr + P;
    const double two_pi = 6.283185307179586476925286766559;
    double r = 0.0, g = 0.0;
    for (int k = threadIdx.x; k < d.nk; k += blockDim.x) {
        const int kx = k / d.nz, kz = k - kx * d.nz;
        const double w = (kx == 0 || 2 * kx == d.nx) ? 1.0 : 2.0;
        const double v = w * s[(size_t)k * d.pstr].x;
        r += v;
        if (a == 0) {
            const int kzs = (kz <= d.nz / 2) ? kz : kz - d.nz;
            const double al = (2 * kx == d.nx) ? 0.0 : two_pi * kx / d.lx;
            const double be = (2 * kz == d.nz) ? 0.0 : two_pi * kzs / d.lz;
            g += (al * al + be * be) * v;
        }
    }
    r = block_sum(r, sh);
    g = block_sum(g, sh);
    if (threadIdx.x == 0) {
        r0[y * 5 + a] = r * inv_count;
        if (a == 0) gxz[y] = g * inv_count;
    }
}

hipError_t launch_r0(hipStream_t st, const Dims &d, const Tables &t, const cx<double> *acc,
                     double inv_count, double *r0, double *gxz)
{
    hipLaunchKernelGGL(k_r0, dim3(d.ny, 5), dim3(256), 0, st, acc, d, t, inv_count, r0, gxz);
    return hipGetLastError();
}

// One block per plane: reduce the per-block partials of the moment kernel;
// eps = nu (<(d_x u')^2 + (d_z u')^2> + <(D u')^2>) with D the five-point
// wall-normal weights: <(D u')^2> = sum_ab w_a w_b <u'(Y_a) u'(Y_b)>.
__global__ void k_profiles(int ny, int nzb, const double *__restrict__ momp,
                           const double *__restrict__ w5, const int *__restrict__ j0,
                           const double *__restrict__ r0, const double *__restrict__ gxz,
                           const double *__restrict__ gy1, double inv_pts, double nu,
                           int gy_mode, double *__restrict__ prof)
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
    double gy = 0.0;
    const int js = j0[j];
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            const int ya = js + a, yb = js + b;
            const int lo = ya < yb ? ya : yb, df = ya < yb ? yb - ya : ya - yb;
            gy += w5[j * 5 + a] * w5[j * 5 + b] * r0[lo * 5 + df];
        }
    prof[P_Q * ny + j] = s[MP_Q];
    prof[P_UV * ny + j] = s[MP_UV];
    prof[P_PV * ny + j] = s[MP_PV];
    prof[P_TX * ny + j] = s[MP_QU];
    prof[P_TY * ny + j] = s[MP_QV];
    prof[P_TZ * ny + j] = s[MP_QW];
    // the split-BF16 path sums the wall-normal part in physical space (FP64):
    // in the first scan (gy1), or in the second (the x pass's stencil) when
    // the caller gave the means
    if (gy_mode == 1) gy = gy1[j];
    else if (gy_mode == 2) gy = s[MP_GY];
    prof[P_EPS * ny + j] = nu * (gy + gxz[j]);
}

hipError_t launch_profiles(hipStream_t st, const Dims &d, const Tables &t, const double *momp,
                           const double *r0, const double *gxz, const double *gy1, int gy_mode,
                           double count, double *prof)
{
    if (gy_mode < 0 || gy_mode > 2 || (gy_mode == 1 && !gy1)) return hipErrorInvalidValue;
    const double inv_pts = 1.0 / (count * (double)d.nx * (double)d.nz);
    hipLaunchKernelGGL(k_profiles, dim3(d.ny), dim3(64), 0, st, d.ny, d.nzb, momp, t.w5, t.j0,
                       r0, gxz, gy1, inv_pts, d.nu, gy_mode, prof);
    return hipGetLastError();
}

// Band accumulators for the general modes (where the accumulators hold only
// the rows of one slab): for every wavenumber k, plane Y and offset a = 0..4,
//   band[k][a][Y] (+)= sum over the chunk of sum_i Re conj(u_i^(k;Y)) u_i^(k;Y+a),
// the same scale-energy products k_r0 reads from the full accumulators.
template <typename S>
__global__ __launch_bounds__(256) void k_band(const S *__restrict__ spec, Dims d, int nsnap,
                                              int accumulate, double *__restrict__ band)
{
    const int k = blockIdx.x, ny = d.ny;
    const S *kb = spec_base(spec, d, k);
    for (int e = threadIdx.x; e < 5 * ny; e += blockDim.x) {
        const int a = e / ny, j = e - a * ny;
        double s = 0.0;
        if (j + a < ny) {
            if constexpr (sizeof(S) == sizeof(SplitRec)) {
                // whole records (four snapshots) per 16-byte load pair
                typedef unsigned int u4v __attribute__((ext_vector_type(4)));
                for (int q = 0; q < (nsnap + 3) >> 2; ++q)
                    for (int f = F_U; f <= F_W; ++f) {
                        const SplitRec *rx = kb + (f * d.nqs + q) * d.nys + j, *ry = rx + a;
                        const u4v xh = *reinterpret_cast<const u4v *>(rx->h);
                        const u4v xl = *reinterpret_cast<const u4v *>(rx->l);
                        const u4v yh = *reinterpret_cast<const u4v *>(ry->h);
                        const u4v yl = *reinterpret_cast<const u4v *>(ry->l);
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (4 * q + t < nsnap) {
                                const cx<double> x = value_of(bf16x4{xh[t], xl[t]});
                                const cx<double> y = value_of(bf16x4{yh[t], yl[t]});
                                s += x.x * y.x + x.y * y.y;
                            }
                        }
                    }
            } else {
                for (int sl = 0; sl < nsnap; ++sl)
                    for (int f = F_U; f <= F_W; ++f) {
                        const cx<double> x = value_of(raw_at(kb, d, f, sl, j));
                        const cx<double> y = value_of(raw_at(kb, d, f, sl, j + a));
                        s += x.x * y.x + x.y * y.y;
                    }
            }
        }
        double *dst = band + (size_t)k * 5 * ny + e;
        *dst = accumulate ? *dst + s : s;
    }
}

hipError_t launch_band(hipStream_t st, const Dims &d, const void *spec, int nsnap,
                       int accumulate, double *band)
{
    if (d.prec == PREC_BF16X3)
        hipLaunchKernelGGL(k_band<SplitRec>, dim3(d.nk), dim3(256), 0, st, (const SplitRec *)spec,
                           d, nsnap, accumulate, band);
    else
        hipLaunchKernelGGL(k_band<cx<double>>, dim3(d.nk), dim3(256), 0, st,
                           (const cx<double> *)spec, d, nsnap, accumulate, band);
    return hipGetLastError();
}

// r0 and gxz of k_r0 from the band accumulators (one block per (Y, a)).
__global__ __launch_bounds__(256) void k_r0_band(const double *__restrict__ band, Dims d,
                                                 double inv_count, double *__restrict__ r0,
                                                 double *__restrict__ gxz)
{
    __shared__ double sh[8];
    const int y = blockIdx.x, a = blockIdx.y, ny = d.ny;
    if (y + a >= ny) {
        if (threadIdx.x == 0) r0[y * 5 + a] = 0.0;
        return;
    }
    const double two_pi = 6.283185307179586476925286766559;
    double r = 0.0, g = 0.0;
    for (int k = threadIdx.x; k < d.nk; k += blockDim.x) {
        const int kx = k / d.nz, kz = k - kx * d.nz;
        const double w = (kx == 0 || 2 * kx == d.nx) ? 1.0 : 2.0;
        const double v = w * band[(size_t)k * 5 * ny + a * ny + y];
        r += v;
        if (a == 0) {
            const int kzs = (kz <= d.nz / 2) ? kz : kz - d.nz;
            const double al = (2 * kx == d.nx) ? 0.0 : two_pi * kx / d.lx;
            const double be = (2 * kz == d.nz) ? 0.0 : two_pi * kzs / d.lz;
            g += (al * al + be * be) * v;
        }
    }
    r = block_sum(r, sh);
    g = block_sum(g, sh);
    if (threadIdx.x == 0) {
        r0[y * 5 + a] = r * inv_count;
        if (a == 0) gxz[y] = g * inv_count;
    }
}

hipError_t launch_r0_band(hipStream_t st, const Dims &d, const double *band, double inv_count,
                          double *r0, double *gxz)
{
    hipLaunchKernelGGL(k_r0_band, dim3(d.ny, 5), dim3(256), 0, st, band, d, inv_count, r0, gxz);
    return hipGetLastError();
}

// Zero n bytes at p (p 8-byte aligned, n a multiple of 8): a plain fill kernel,
// so that clearing never records a memset node in a caller's captured graph.
__global__ __launch_bounds__(256) void k_zero(unsigned long long *__restrict__ p, size_t n8)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_zero(hipStream_t st, void *p, size_t bytes)
{
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)p & 7) || (bytes & 7)) return hipErrorInvalidValue;
    const size_t n8 = bytes >> 3;
    const unsigned nb = (unsigned)std::min<size_t>((n8 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(nb), dim3(256), 0, st, (unsigned long long *)p, n8);
    return hipGetLastError();
}

__global__ void k_t14(int ny, const double *__restrict__ prof, void *__restrict__ t14, int f32)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ny * ny) return;
    const int j1 = i / ny, j2 = i - j1 * ny;
    // -4 <eps*>, eps* the average of the two points
    const double v = -2.0 * (prof[P_EPS * ny + j1] + prof[P_EPS * ny + j2]);
    if (f32) static_cast<float *>(t14)[i] = (float)v;
    else static_cast<double *>(t14)[i] = v;
}

hipError_t launch_t14(hipStream_t st, const Dims &d, const double *prof, void *t14, int f32)
{
    const int n = d.ny * d.ny;
    hipLaunchKernelGGL(k_t14, dim3((n + 255) / 256), dim3(256), 0, st, d.ny, prof, t14, f32);
    return hipGetLastError();
}

}  // namespace gke
