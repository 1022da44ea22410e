// k_step1.hip -- Step 1 upstream of the statistics (Section "Step 1": when
// the database holds only the wall-normal velocity and vorticity, as Fourier
// coefficients in x and z, the full velocity is computed, and the pressure is
// obtained from its Poisson equation for each velocity field).
//
// Coefficients f^(kx, kz; y) over the half spectrum, f = sum_k f^ e^{i k.x}
// (the forward transform scaled by 1/(Nx Nz)), layout [Ny][Nz][Nx/2 + 1];
// alpha, beta with zero multipliers at the Nyquist wavenumbers.
//   velocity: continuity i alpha u^ + D v^ + i beta w^ = 0 and
//     omega^ = i beta u^ - i alpha w^ give, for k^2 > 0,
//     u^ = i (alpha D v^ - beta omega^) / k^2, w^ = i (beta D v^ + alpha omega^) / k^2;
//     the (0, 0) mode of u, w is the given plane-mean profile;
//   pressure: lap p = -d_i d_j (u_i u_j) with the products of the total
//     velocity formed on the grid; per wavenumber on the interior nodes
//     (D2 - k^2) p^ = alpha^2 uu^ + 2 alpha beta uw^ + beta^2 ww^
//                     - 2 i alpha D uv^ - 2 i beta D vw^ - D2 vv^,
//     at the walls D p^ = nu D2 v^ (wall-normal momentum with no slip); the
//     (0, 0) mode p^ = -vv^; other bins with k^2 = 0 carry no pressure.
// D: the five-point first derivative of Step 3; D2: five-point second
// derivative weights on the same windows.
#include <algorithm>

#include "gke_internal.h"

namespace gke {

template <typename F>
static void set_lds_limit_s1(F *kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)LDS_BUDGET);
}

__device__ __forceinline__ double alpha_of(const Dims &d, int kx)
{
    return (2 * kx == d.nx) ? 0.0 : 6.283185307179586476925286766559 * kx / d.lx;
}
__device__ __forceinline__ double beta_of(const Dims &d, int kz)
{
    const int ks = (kz <= d.nz / 2) ? kz : kz - d.nz;
    return (2 * kz == d.nz) ? 0.0 : 6.283185307179586476925286766559 * ks / d.lz;
}

// Velocity spectra: one thread per (plane j, wavenumber k); vel = [u^, v^, w^].
__global__ __launch_bounds__(256) void k_s1_vel(const cx<double> *__restrict__ vh,
                                                const cx<double> *__restrict__ oh,
                                                const double *__restrict__ mean_u,
                                                const double *__restrict__ mean_w, Dims d,
                                                Tables t, cx<double> *__restrict__ vel)
{
    const size_t nk = d.nk, plane = (size_t)d.ny * nk;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= plane) return;
    const int j = (int)(e / nk), k = (int)(e - (size_t)j * nk);
    const int kz = k / d.nkx, kx = k - kz * d.nkx;
    const cx<double> v = vh[e];
    if (k == 0) {
        vel[e] = cx<double>{mean_u[j], 0.0};
        vel[plane + e] = v;
        vel[2 * plane + e] = cx<double>{mean_w[j], 0.0};
        return;
    }
    const int j0 = t.j0[j];
    cx<double> dv{0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const cx<double> x = vh[(size_t)(j0 + a) * nk + k];
        const double wt = t.w5[j * 5 + a];
        dv.x += wt * x.x;
        dv.y += wt * x.y;
    }
    const cx<double> om = oh[e];
    const double al = alpha_of(d, kx), be = beta_of(d, kz), k2 = al * al + be * be;
    cx<double> u{0.0, 0.0}, w{0.0, 0.0};
    if (k2 > 0.0) {
        // i (alpha dv - beta om) / k2 and i (beta dv + alpha om) / k2
        const double ar = (al * dv.x - be * om.x) / k2, ai = (al * dv.y - be * om.y) / k2;
        const double br = (be * dv.x + al * om.x) / k2, bi = (be * dv.y + al * om.y) / k2;
        u = cx<double>{-ai, ar};
        w = cx<double>{-bi, br};
    }
    vel[e] = u;
    vel[plane + e] = v;
    vel[2 * plane + e] = w;
}

// Transforms along z of the half-spectrum planes of nf fields, in place:
// block = kb consecutive kx of one (plane, field); batch of kb transforms of
// length Nz in LDS; sign +1 inverse (unscaled), -1 forward scaled by `scale`.
__global__ GKE_FFT_BOUNDS void k_s1_zfft(cx<double> *__restrict__ buf, Dims d, Tables t,
                                         int kb, int sign, double scale)
{
    extern __shared__ cx<double> lds[];
    const int nz = d.nz, nkx = d.nkx;
    const int kx0 = blockIdx.x * kb, j = blockIdx.y, f = blockIdx.z;
    const int nb = min(kb, nkx - kx0);
    const int bs = fft_stride(nz);
    cx<double> *tw = lds + kb * bs;
    cx<double> *base = buf + ((size_t)f * d.ny + j) * (size_t)nz * nkx + kx0;
    {
        TwiddleCopy<double, FFT_BLOCK> twc;
        twc.load(t.twz, nz);
        twc.store(tw, t.twz, nz);
    }
    for (int e = threadIdx.x; e < nz * nb; e += FFT_BLOCK) {
        const int kz = e / nb, b = e - kz * nb;
        lds[b * bs + fft_pad(kz)] = base[(size_t)kz * nkx + b];
    }
    __syncthreads();
    lds_fft_ip<double, FFT_CAP, FFT_BLOCK>(lds, nb, bs, t.pz, tw, sign);
    for (int e = threadIdx.x; e < nz * nb; e += FFT_BLOCK) {
        const int kz = e / nb, b = e - kz * nb;
        base[(size_t)kz * nkx + b] = cscale(lds[b * bs + fft_pad(kz)], scale);
    }
}

// Inverse real transforms along x of kz-transformed half-spectrum rows, two
// rows (z, z + 1) per complex transform: A[kx] = X1[kx] + i X2[kx],
// A[Nx - kx] = conj X1[kx] + i conj X2[kx], and at kx = 0, Nx/2 the real parts
// (the values of real fields); Re and Im of the inverse are the two rows.
// Block = nr row pairs of one (plane, field); out[f] are [Ny][Nz][Nx] arrays.
struct S1Out {
    double *f[4];
};
__global__ GKE_FFT_BOUNDS void k_s1_xinv(const cx<double> *__restrict__ buf, Dims d, Tables t,
                                         int nr, int f0, S1Out out)
{
    extern __shared__ cx<double> lds[];
    const int nx = d.nx, nz = d.nz, nkx = d.nkx;
    const int c0 = blockIdx.x * nr, j = blockIdx.y, f = blockIdx.z;
    const int nc = min(nr, nz / 2 - c0);
    const int bs = fft_stride(nx);
    cx<double> *tw = lds + nr * bs;
    const cx<double> *base = buf + ((size_t)(f0 + f) * d.ny + j) * (size_t)nz * nkx;
    {
        TwiddleCopy<double, FFT_BLOCK> twc;
        twc.load(t.twx, nx);
        twc.store(tw, t.twx, nx);
    }
    for (int e = threadIdx.x; e < nkx * nc; e += FFT_BLOCK) {
        const int c = e / nkx, kx = e - c * nkx;
        const int z = 2 * (c0 + c);
        const cx<double> a = base[(size_t)z * nkx + kx], b = base[(size_t)(z + 1) * nkx + kx];
        cx<double> *A = lds + c * bs;
        if (kx == 0 || 2 * kx == nx) {
            A[fft_pad(kx)] = cx<double>{a.x, b.x};
        } else {
            A[fft_pad(kx)] = cx<double>{a.x - b.y, a.y + b.x};
            A[fft_pad(nx - kx)] = cx<double>{a.x + b.y, b.x - a.y};
        }
    }
    __syncthreads();
    lds_fft_ip<double, FFT_CAP, FFT_BLOCK>(lds, nc, bs, t.px, tw, +1);
    double *o = out.f[f] + (size_t)j * nz * nx;
    for (int e = threadIdx.x; e < nx * nc; e += FFT_BLOCK) {
        const int c = e / nx, x = e - c * nx;
        const int z = 2 * (c0 + c);
        const cx<double> v = lds[c * bs + fft_pad(x)];
        o[(size_t)z * nx + x] = v.x;
        o[(size_t)(z + 1) * nx + x] = v.y;
    }
}

// Products of the total velocity and their forward transforms along x:
// block = nr z rows of one plane; per row the six products uu uw ww uv vw vv
// packed two per complex transform, unpacked as F[k] = (A[k] + conj A[-k])/2,
// G[k] = (A[k] - conj A[-k])/(2i), scaled by 1/(Nx Nz), into
// prod[6][Ny][Nz][Nkx] (the z transform follows).
__global__ GKE_FFT_BOUNDS void k_s1_prod_x(const double *__restrict__ u,
                                           const double *__restrict__ v,
                                           const double *__restrict__ w, Dims d, Tables t,
                                           int nr, cx<double> *__restrict__ prod)
{
    extern __shared__ cx<double> lds[];
    const int nx = d.nx, nz = d.nz, nkx = d.nkx;
    const int z0 = blockIdx.x * nr, j = blockIdx.y;
    const int nc = min(nr, nz - z0);
    const int bs = fft_stride(nx);
    cx<double> *tw = lds + 3 * nr * bs;
    {
        TwiddleCopy<double, FFT_BLOCK> twc;
        twc.load(t.twx, nx);
        twc.store(tw, t.twx, nx);
    }
    const size_t row0 = ((size_t)j * nz + z0) * nx;
    for (int e = threadIdx.x; e < nx * nc; e += FFT_BLOCK) {
        const int c = e / nx, x = e - c * nx;
        const size_t o = row0 + (size_t)c * nx + x;
        const double a = u[o], b = v[o], q = w[o];
        lds[(3 * c + 0) * bs + fft_pad(x)] = cx<double>{a * a, a * q};   // uu, uw
        lds[(3 * c + 1) * bs + fft_pad(x)] = cx<double>{q * q, a * b};   // ww, uv
        lds[(3 * c + 2) * bs + fft_pad(x)] = cx<double>{b * q, b * b};   // vw, vv
    }
    __syncthreads();
    lds_fft_ip<double, FFT_CAP, FFT_BLOCK>(lds, 3 * nc, bs, t.px, tw, -1);
    const double s = 1.0 / ((double)nx * (double)nz);
    const size_t fstride = (size_t)d.ny * nz * nkx;
    for (int e = threadIdx.x; e < nkx * nc; e += FFT_BLOCK) {
        const int c = e / nkx, kx = e - c * nkx;
        const int kn = kx == 0 ? 0 : nx - kx;
        const size_t o = ((size_t)j * nz + z0 + c) * nkx + kx;
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            const cx<double> A = lds[(3 * c + g) * bs + fft_pad(kx)];
            const cx<double> B = lds[(3 * c + g) * bs + fft_pad(kn)];   // A[-k]
            // F = (A + conj B)/2, G = (A - conj B)/(2i)
            const cx<double> F{0.5 * (A.x + B.x), 0.5 * (A.y - B.y)};
            const cx<double> G{0.5 * (A.y + B.y), -0.5 * (A.x - B.x)};
            prod[(size_t)(2 * g) * fstride + o] = cscale(F, s);
            prod[(size_t)(2 * g + 1) * fstride + o] = cscale(G, s);
        }
    }
}

// Pressure per wavenumber: one thread per k.  The banded system (rows of the
// five-point windows: lower and upper bandwidth 4) is eliminated with partial
// pivoting over a sliding window of five rows by nine columns held in
// registers; the pivot rows go to the scratch U [Ny][9][nk], B [Ny][nk], then
// back substitution writes p^ [Ny][Nz][Nkx].
enum { PR_UU = 0, PR_UW, PR_WW, PR_UV, PR_VW, PR_VV };
__global__ __launch_bounds__(256) void k_s1_press(const cx<double> *__restrict__ prod,
                                                  const cx<double> *__restrict__ vh, Dims d,
                                                  Tables t, double *__restrict__ su,
                                                  cx<double> *__restrict__ sb,
                                                  cx<double> *__restrict__ ph)
{
    const int nk = d.nk, ny = d.ny;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    const size_t fs = (size_t)ny * nk;
    auto P = [&](int f, int j) { return prod[(size_t)f * fs + (size_t)j * nk + k]; };
    if (k == 0) {   // the (0, 0) mode
        for (int j = 0; j < ny; ++j) {
            const cx<double> vv = P(PR_VV, j);
            ph[(size_t)j * nk] = cx<double>{-vv.x, -vv.y};
        }
        return;
    }
    const int kz = k / d.nkx, kx = k - kz * d.nkx;
    const double al = alpha_of(d, kx), be = beta_of(d, kz), k2 = al * al + be * be;
    if (!(k2 > 0.0)) {
        for (int j = 0; j < ny; ++j) ph[(size_t)j * nk + k] = cx<double>{0.0, 0.0};
        return;
    }
    // row r of the system into coefficients c[0..8] for columns c0 .. c0 + 8
    // and its right-hand side
    // (the coefficients are placed by selects on the static column index, so
    // that the window stays in registers)
    auto place = [](double *c, const double *wv, int off) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) s = (q == off + a) ? wv[a] : s;
            c[q] = s;
        }
    };
    auto build = [&](int r, int c0, double *c, cx<double> &rhs) {
        const int j0 = t.j0[r];
        const int off = j0 - c0;   // 0 .. 2 (see the window argument below)
        double wv[5];
        if (r == 0 || r == ny - 1) {
            // wall rows: D p = nu D2 v
            cx<double> s{0.0, 0.0};
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                wv[a] = t.w5[r * 5 + a];
                const cx<double> x = vh[(size_t)(j0 + a) * nk + k];
                s.x += t.w2[r * 5 + a] * x.x;
                s.y += t.w2[r * 5 + a] * x.y;
            }
            place(c, wv, off);
            rhs = cx<double>{d.nu * s.x, d.nu * s.y};
            return;
        }
        cx<double> duv{0.0, 0.0}, dvw{0.0, 0.0}, d2vv{0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const double w1 = t.w5[r * 5 + a], w2 = t.w2[r * 5 + a];
            wv[a] = w2;
            const cx<double> uv = P(PR_UV, j0 + a), vw = P(PR_VW, j0 + a), vv = P(PR_VV, j0 + a);
            duv.x += w1 * uv.x; duv.y += w1 * uv.y;
            dvw.x += w1 * vw.x; dvw.y += w1 * vw.y;
            d2vv.x += w2 * vv.x; d2vv.y += w2 * vv.y;
        }
        place(c, wv, off);
#pragma unroll
        for (int q = 0; q < 9; ++q) c[q] -= (q == r - c0) ? k2 : 0.0;
        const cx<double> uu = P(PR_UU, r), uw = P(PR_UW, r), ww = P(PR_WW, r);
        // alpha^2 uu + 2 alpha beta uw + beta^2 ww - 2 i (alpha duv + beta dvw) - d2vv
        const double ra = al * al, rb = 2.0 * al * be, rc = be * be;
        const cx<double> g{2.0 * (al * duv.x + be * dvw.x), 2.0 * (al * duv.y + be * dvw.y)};
        rhs = cx<double>{ra * uu.x + rb * uw.x + rc * ww.x + g.y - d2vv.x,
                         ra * uu.y + rb * uw.y + rc * ww.y - g.x - d2vv.y};
    };
    // The window holds the rows j .. j + 4 over the columns j .. j + 8.  An
    // original row r enters when the window starts at c0 = r - 4 (r >= 5) or
    // at 0 (r < 5); its five nodes j0[r] .. j0[r] + 4 lie in that range.
    double c[5][9];
    cx<double> b[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        if (r < ny) build(r, 0, c[r], b[r]);
        else {
#pragma unroll
            for (int q = 0; q < 9; ++q) c[r][q] = 0.0;
            b[r] = cx<double>{0.0, 0.0};
        }
    }
    for (int j = 0; j < ny; ++j) {
        // partial pivoting: the largest |c[r][0]| to row 0
#pragma unroll
        for (int r = 1; r < 5; ++r) {
            const bool sw = fabs(c[r][0]) > fabs(c[0][0]);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double a0 = c[0][q], ar = c[r][q];
                c[0][q] = sw ? ar : a0;
                c[r][q] = sw ? a0 : ar;
            }
            const cx<double> b0 = b[0], br = b[r];
            b[0] = sw ? br : b0;
            b[r] = sw ? b0 : br;
        }
        const double inv = 1.0 / c[0][0];
#pragma unroll
        for (int r = 1; r < 5; ++r) {
            const double m = c[r][0] * inv;
#pragma unroll
            for (int q = 0; q < 9; ++q) c[r][q] -= m * c[0][q];
            b[r].x -= m * b[0].x;
            b[r].y -= m * b[0].y;
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) su[((size_t)j * 9 + q) * nk + k] = c[0][q];
        sb[(size_t)j * nk + k] = b[0];
        // shift the window one row down and one column right, then enter row j + 5
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int q = 0; q < 8; ++q) c[r][q] = c[r + 1][q + 1];
            c[r][8] = 0.0;
            b[r] = b[r + 1];
        }
        if (j + 5 < ny) build(j + 5, j + 1, c[4], b[4]);
        else {
#pragma unroll
            for (int q = 0; q < 9; ++q) c[4][q] = 0.0;
            b[4] = cx<double>{0.0, 0.0};
        }
    }
    // back substitution with the last eight solution values in registers
    cx<double> xs[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xs[q] = cx<double>{0.0, 0.0};
    for (int j = ny - 1; j >= 0; --j) {
        cx<double> s = sb[(size_t)j * nk + k];
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            const double u = su[((size_t)j * 9 + q) * nk + k];
            s.x -= u * xs[q - 1].x;
            s.y -= u * xs[q - 1].y;
        }
        const double inv = 1.0 / su[((size_t)j * 9) * nk + k];
        const cx<double> x{s.x * inv, s.y * inv};
#pragma unroll
        for (int q = 7; q > 0; --q) xs[q] = xs[q - 1];
        xs[0] = x;
        ph[(size_t)j * nk + k] = x;
    }
}

hipError_t launch_step1(hipStream_t st, const Dims &d, const Tables &t, const cx<double> *vh,
                        const cx<double> *oh, const double *mean_u, const double *mean_w,
                        cx<double> *vel, cx<double> *prod, cx<double> *ph, double *su,
                        cx<double> *sb, double *u, double *v, double *w, double *p)
{
    const size_t npts = (size_t)d.ny * d.nk;
    hipLaunchKernelGGL(k_s1_vel, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, vh, oh,
                       mean_u, mean_w, d, t, vel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // transform shapes: kb kx columns (z passes), nr row pairs / rows (x passes)
    const int sz = fft_stride(d.nz), sx = fft_stride(d.nx);
    const int capz = FFT_CAP / sz, capx = FFT_CAP / sx;
    const int kb = std::max(1, std::min(std::min(16, capz), d.nkx));
    const int nr = std::max(1, std::min(std::min(8, capx), d.nz / 2));
    const int nr3 = std::max(1, std::min(8, capx / 3));
    if (capz < 1 || capx < 3) return hipErrorInvalidValue;
    const size_t ldsz = sizeof(cx<double>) * ((size_t)kb * sz + d.nz);
    const size_t ldsx = sizeof(cx<double>) * ((size_t)nr * sx + d.nx);
    const size_t ldsp = sizeof(cx<double>) * ((size_t)3 * nr3 * sx + d.nx);
    set_lds_limit_s1(k_s1_zfft);
    set_lds_limit_s1(k_s1_xinv);
    set_lds_limit_s1(k_s1_prod_x);
    // velocity to physical space
    hipLaunchKernelGGL(k_s1_zfft, dim3((d.nkx + kb - 1) / kb, d.ny, 3), dim3(FFT_BLOCK), ldsz, st,
                       vel, d, t, kb, +1, 1.0);
    S1Out ov{{u, v, w, nullptr}};
    hipLaunchKernelGGL(k_s1_xinv, dim3((d.nz / 2 + nr - 1) / nr, d.ny, 3), dim3(FFT_BLOCK), ldsx,
                       st, vel, d, t, nr, 0, ov);
    // products and their spectra
    hipLaunchKernelGGL(k_s1_prod_x, dim3((d.nz + nr3 - 1) / nr3, d.ny), dim3(FFT_BLOCK), ldsp, st,
                       u, v, w, d, t, nr3, prod);
    hipLaunchKernelGGL(k_s1_zfft, dim3((d.nkx + kb - 1) / kb, d.ny, 6), dim3(FFT_BLOCK), ldsz, st,
                       prod, d, t, kb, -1, 1.0);
    // pressure spectrum, then physical space
    hipLaunchKernelGGL(k_s1_press, dim3((d.nk + 255) / 256), dim3(256), 0, st, prod, vh, d, t, su,
                       sb, ph);
    hipLaunchKernelGGL(k_s1_zfft, dim3((d.nkx + kb - 1) / kb, d.ny, 1), dim3(FFT_BLOCK), ldsz, st,
                       ph, d, t, kb, +1, 1.0);
    S1Out op{{p, nullptr, nullptr, nullptr}};
    hipLaunchKernelGGL(k_s1_xinv, dim3((d.nz / 2 + nr - 1) / nr, d.ny, 1), dim3(FFT_BLOCK), ldsx,
                       st, ph, d, t, nr, 0, op);
    return hipGetLastError();
}

}  // namespace gke
