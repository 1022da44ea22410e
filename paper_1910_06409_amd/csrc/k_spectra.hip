// k_spectra.hip -- per-snapshot part of the second scan (Section "Step 2"):
// fluctuations about the Step-1 means (FP64), the in-plane products formed in
// physical space (Section "Products instead of correlations"), and the 2-D
// forward transform of every plane, written in the layout the cross-spectral
// update reads.  Also the FP64 one-point moments and the pseudo-dissipation
// pieces (x and z derivatives spectral, y derivative by the five-point
// stencil).
//
// Normalisation: A^(kx,kz) = (1/(Nx Nz)) sum_{x,z} A e^{-i(alpha x + beta z)}.
#include "gke_internal.h"

namespace gke {

__device__ __forceinline__ double field_value(int f, double a, double b, double c, double d)
{
    switch (f) {
    case F_U: return a;
    case F_V: return b;
    case F_W: return c;
    case F_P: return d;
    case F_UU: return a * a;
    case F_VV: return b * b;
    case F_WW: return c * c;
    case F_UV: return a * b;
    case F_UW: return a * c;
    default: return b * c;  // F_VW
    }
}

__device__ __forceinline__ double block_sum256(double v, double *sh)
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

// One block = zb consecutive z rows of plane j.
//   inter[j][f][kx][z]: x-transformed rows (unnormalised) of the ten fields
//   momp[j][k][zblk]: FP64 partial sums of q uv pv qu qv qw and (dy u')^2
template <typename TI>
__global__ __launch_bounds__(256) void k_fluct_xfft(const TI *__restrict__ u,
                                                    const TI *__restrict__ v,
                                                    const TI *__restrict__ w,
                                                    const TI *__restrict__ p,
                                                    const double *__restrict__ prof, Dims d,
                                                    Tables t, cx<double> *__restrict__ inter,
                                                    double *__restrict__ momp)
{
    extern __shared__ cx<double> lds[];
    __shared__ double sh[8];
    const int nx = d.nx, ny = d.ny, nz = d.nz, nkx = d.nkx, zb = d.zb;
    const int zblk = blockIdx.x, j = blockIdx.y;
    const int z0 = zblk * zb;
    const int bs = nx + 1;
    cx<double> *A = lds;
    cx<double> *B = lds + zb * bs;
    const size_t npl = (size_t)nx * nz;
    const size_t off = (size_t)j * npl + (size_t)z0 * nx;
    const double U = prof[P_U * ny + j], V = prof[P_V * ny + j];
    const double W = prof[P_W * ny + j], P = prof[P_P * ny + j];
    const int nel = zb * nx;

    // one-point moments and the wall-normal gradient energy (FP64)
    {
        const int js = t.j0[j];
        double wt[5], Ms[3][5];
        for (int a = 0; a < 5; ++a) {
            wt[a] = t.w5[j * 5 + a];
            Ms[0][a] = prof[P_U * ny + js + a];
            Ms[1][a] = prof[P_V * ny + js + a];
            Ms[2][a] = prof[P_W * ny + js + a];
        }
        double mq = 0, muv = 0, mpv = 0, mqu = 0, mqv = 0, mqw = 0, mgy = 0;
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            const double a = (double)u[off + e] - U, b = (double)v[off + e] - V;
            const double c = (double)w[off + e] - W, dd = (double)p[off + e] - P;
            const double q = a * a + b * b + c * c;
            mq += q;
            muv += a * b;
            mpv += dd * b;
            mqu += q * a;
            mqv += q * b;
            mqw += q * c;
            double gu = 0, gv = 0, gw = 0;
            for (int k = 0; k < 5; ++k) {
                const size_t o = (size_t)(js + k) * npl + (size_t)z0 * nx + e;
                gu += wt[k] * ((double)u[o] - Ms[0][k]);
                gv += wt[k] * ((double)v[o] - Ms[1][k]);
                gw += wt[k] * ((double)w[o] - Ms[2][k]);
            }
            mgy += gu * gu + gv * gv + gw * gw;
        }
        const double parts[NMOMP] = {mq, muv, mpv, mqu, mqv, mqw, mgy};
        for (int k = 0; k < NMOMP; ++k) {
            const double r = block_sum256(parts[k], sh);
            if (threadIdx.x == 0) momp[((size_t)j * NMOMP + k) * d.nzb + zblk] += r;
        }
    }

    // five complex pairs of real fields: (u,v) (w,p) (uu,vv) (ww,uv) (uw,vw)
    for (int pr = 0; pr < NFIELD / 2; ++pr) {
        const int fa = 2 * pr, fb = 2 * pr + 1;
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
            const double a = (double)u[off + e] - U, b = (double)v[off + e] - V;
            const double c = (double)w[off + e] - W, dd = (double)p[off + e] - P;
            const int row = e / nx, x = e - row * nx;
            A[row * bs + x] = cx<double>{field_value(fa, a, b, c, dd), field_value(fb, a, b, c, dd)};
        }
        __syncthreads();
        const cx<double> *R = lds_fft<double>(A, B, zb, bs, t.px, t.twx, -1);
        // split the two real transforms: Fa = (Z(k) + conj Z(-k))/2, Fb = (Z(k) - conj Z(-k))/(2i)
        for (int e = threadIdx.x; e < nkx * zb; e += blockDim.x) {
            const int k = e / zb, row = e - k * zb;
            const cx<double> Z = R[row * bs + k];
            const cx<double> Zc = cconj(R[row * bs + (k == 0 ? 0 : nx - k)]);
            const cx<double> Fa = cx<double>{0.5 * (Z.x + Zc.x), 0.5 * (Z.y + Zc.y)};
            const cx<double> Fb = cx<double>{0.5 * (Z.y - Zc.y), -0.5 * (Z.x - Zc.x)};
            inter[(((size_t)j * NFIELD + fa) * nkx + k) * nz + z0 + row] = Fa;
            inter[(((size_t)j * NFIELD + fb) * nkx + k) * nz + z0 + row] = Fb;
        }
        __syncthreads();
    }
}

hipError_t launch_fluct_xfft(hipStream_t st, const Dims &d, const Tables &t, int f32,
                             const void *u, const void *v, const void *w, const void *p,
                             const double *prof, cx<double> *inter, double *momp)
{
    const size_t lds = sizeof(cx<double>) * 2 * (size_t)d.zb * (d.nx + 1);
    dim3 grid(d.nzb, d.ny);
    if (f32)
        hipLaunchKernelGGL(k_fluct_xfft<float>, grid, dim3(256), lds, st, (const float *)u,
                           (const float *)v, (const float *)w, (const float *)p, prof, d, t,
                           inter, momp);
    else
        hipLaunchKernelGGL(k_fluct_xfft<double>, grid, dim3(256), lds, st, (const double *)u,
                           (const double *)v, (const double *)w, (const double *)p, prof, d, t,
                           inter, momp);
    return hipGetLastError();
}

// One block = jb consecutive planes of one field at one kx: transform along z,
// scale, and store spec[k = kx*Nz + kz][f][slot][j] (planes contiguous).
// For u, v, w also add sum_kz w_kx (alpha^2 + beta^2)|A^|^2 into momg[j][f][kx]
// (the plane average of (dx u')^2 + (dz u')^2 by the Parseval identity).
__global__ __launch_bounds__(256) void k_zfft_pack(const cx<double> *__restrict__ inter, Dims d,
                                                   Tables t, int slot,
                                                   cx<double> *__restrict__ spec,
                                                   double *__restrict__ momg)
{
    extern __shared__ cx<double> lds[];
    __shared__ double red[256];
    const int nx = d.nx, ny = d.ny, nz = d.nz, nkx = d.nkx, jb = d.jb;
    const int jblk = blockIdx.x, kx = blockIdx.y, f = blockIdx.z;
    const int j0 = jblk * jb;
    const int nb = min(jb, ny - j0);
    const int bs = nz + 1;
    cx<double> *A = lds;
    cx<double> *B = lds + jb * bs;
    for (int e = threadIdx.x; e < nb * nz; e += blockDim.x) {
        const int b = e / nz, z = e - b * nz;
        A[b * bs + z] = inter[(((size_t)(j0 + b) * NFIELD + f) * nkx + kx) * nz + z];
    }
    __syncthreads();
    const cx<double> *R = lds_fft<double>(A, B, nb, bs, t.pz, t.twz, -1);
    const double scale = 1.0 / ((double)nx * (double)nz);
    const double two_pi = 6.283185307179586476925286766559;
    const double alpha = (2 * kx == nx) ? 0.0 : two_pi * kx / d.lx;
    const double wkx = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
    double eg = 0.0;
    for (int e = threadIdx.x; e < jb * nz; e += blockDim.x) {
        const int kz = e / jb, b = e - kz * jb;
        if (b < nb) {
            const cx<double> X = cscale(R[b * bs + kz], scale);
            spec[((((size_t)kx * nz + kz) * NFIELD + f) * d.chunk + slot) * ny + j0 + b] = X;
            if (f < 3) {
                const int kzs = (kz <= nz / 2) ? kz : kz - nz;
                const double beta = (2 * kz == nz) ? 0.0 : two_pi * kzs / d.lz;
                eg += wkx * (alpha * alpha + beta * beta) * (X.x * X.x + X.y * X.y);
            }
        }
    }
    if (f < 3) {
        // every thread works on one plane b = threadIdx.x % jb (blockDim % jb == 0)
        red[threadIdx.x] = eg;
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            double s = 0.0;
            for (int i = threadIdx.x; i < (int)blockDim.x; i += jb) s += red[i];
            momg[((size_t)(j0 + threadIdx.x) * 3 + f) * nkx + kx] += s;
        }
    }
}

hipError_t launch_zfft_pack(hipStream_t st, const Dims &d, const Tables &t,
                            const cx<double> *inter, int slot, cx<double> *spec, double *momg)
{
    const size_t lds = sizeof(cx<double>) * 2 * (size_t)d.jb * (d.nz + 1);
    dim3 grid((d.ny + d.jb - 1) / d.jb, d.nkx, NFIELD);
    hipLaunchKernelGGL(k_zfft_pack, grid, dim3(256), lds, st, inter, d, t, slot, spec, momg);
    return hipGetLastError();
}

}  // namespace gke
