// k_final.hip -- end of Step 2 and Step 3 (Sections "Step 2", "Step 3"):
// average over the snapshots, inverse transforms of the term spectra into
// (rx, rz) maps, FP64 assembly with the one-point profiles, and the
// five-point wall-normal derivatives of <du^2>.
//
// Correlation convention: C[A,B](r; Y1, Y2) = sum_k conj(A^(k;Y1)) B^(k;Y2) e^{+i k.r}
// over the full spectrum; the stored half spectrum kx = 0..Nx/2 is extended by
// Hermitian symmetry (the fields are real).  Viscous fluxes in rx and rz are
// spectral derivatives of <du^2> in r (Section "General structure of the
// program"); with <du^2> = <q>(Y1) + <q>(Y2) - 2 R they are 4 nu F^-1(i alpha R^)
// and 4 nu F^-1(i beta R^), with zero multipliers at the Nyquist wavenumbers.
#include <algorithm>

#include "gke_internal.h"

namespace gke {

// Inverse transform along kz for PB pairs of one term spectrum at one kx.
// mid layout: [NMAP][nkx][nz (rz)][ptot (pairs of this batch)].
__global__ __launch_bounds__(256) void k_fin_kz(const cx<double> *__restrict__ acc, Dims d,
                                                Tables t, int p0, int ptot, int pb,
                                                double inv_count, cx<double> *__restrict__ mid)
{
    extern __shared__ cx<double> lds[];
    const int nz = d.nz, nkx = d.nkx;
    const int pblk = blockIdx.x, kx = blockIdx.y, sp = blockIdx.z;
    const int pl0 = pblk * pb;                       // first pair within the batch
    const int np = min(pb, ptot - pl0);
    const size_t pall = (size_t)d.npair;
    const size_t pg0 = (size_t)p0 + pl0;             // first pair within acc
    const int bs = nz + 1;
    cx<double> *A = lds;
    cx<double> *B = lds + pb * bs;
    const double two_pi = 6.283185307179586476925286766559;
    const double alpha = (2 * kx == d.nx) ? 0.0 : two_pi * kx / d.lx;
    const int nout_tr = (sp == S_R) ? 2 : 1;
    for (int tr = 0; tr < nout_tr; ++tr) {
        for (int e = threadIdx.x; e < nz * pb; e += blockDim.x) {
            const int kz = e / pb, b = e - kz * pb;
            if (b < np) {
                cx<double> X = cscale(acc[((size_t)sp * d.nk + (size_t)kx * nz + kz) * pall + pg0 + b],
                                      inv_count);
                if (tr == 1) {  // i beta R^
                    const int kzs = (kz <= nz / 2) ? kz : kz - nz;
                    const double beta = (2 * kz == nz) ? 0.0 : two_pi * kzs / d.lz;
                    X = cx<double>{-beta * X.y, beta * X.x};
                }
                A[b * bs + kz] = X;
            }
        }
        __syncthreads();
        const cx<double> *R = lds_fft<double>(A, B, np, bs, t.pz, t.twz, +1);
        int m0;
        if (sp == S_R) m0 = (tr == 0) ? M_R : M_DRZ;
        else m0 = M_FX + (sp - S_FX);  // FX FY FZ PHI PP UVS UVA map one to one
        for (int e = threadIdx.x; e < nz * pb; e += blockDim.x) {
            const int rz = e / pb, b = e - rz * pb;
            if (b < np) {
                const cx<double> Y = R[b * bs + rz];
                const size_t o = ((size_t)kx * nz + rz) * ptot + pl0 + b;
                mid[(size_t)m0 * nkx * nz * ptot + o] = Y;
                if (sp == S_R && tr == 0)  // i alpha R^: alpha is constant along kz
                    mid[(size_t)M_DRX * nkx * nz * ptot + o] = cx<double>{-alpha * Y.y, alpha * Y.x};
            }
        }
        __syncthreads();
    }
}

hipError_t launch_fin_kz(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *acc, int p0, int p1, double inv_count,
                         cx<double> *mid)
{
    const int ptot = p1 - p0;
    int pb = 8;
    while (pb > 1 && sizeof(cx<double>) * 2 * (size_t)pb * (d.nz + 1) > 65536) pb >>= 1;
    const size_t lds = sizeof(cx<double>) * 2 * (size_t)pb * (d.nz + 1);
    dim3 grid((ptot + pb - 1) / pb, d.nkx, NSPEC);
    hipLaunchKernelGGL(k_fin_kz, grid, dim3(256), lds, st, acc, d, t, p0, ptot, pb, inv_count,
                       mid);
    return hipGetLastError();
}

struct OutPtrs {
    double *t[14];
};

// sign of each map under r-inversion: map(r; Y2, Y1) = sigma * map(-r; Y1, Y2)
__device__ __forceinline__ double map_sigma(int m)
{
    switch (m) {
    case M_R: case M_PHI: case M_PP: case M_UVS: return 1.0;
    default: return -1.0;
    }
}

// Assemble the terms that use map m at (j1, j2) and store them at index o.
__device__ __forceinline__ void assemble_store(int m, double val, int j1, int j2,
                                               const double *prof, int ny, double nu,
                                               const OutPtrs &out, size_t o)
{
#define PR(row, j) prof[(row) * ny + (j)]
    switch (m) {
    case M_R: {
        const double t1 = PR(P_Q, j1) + PR(P_Q, j2) - 2.0 * val;       // <du^2>
        if (out.t[0]) out.t[0][o] = t1;
        if (out.t[2]) out.t[2][o] = (PR(P_U, j2) - PR(P_U, j1)) * t1;  // <du^2 dU>
        break;
    }
    case M_DRX:
        if (out.t[3]) out.t[3][o] = 4.0 * nu * val;
        break;
    case M_DRZ:
        if (out.t[7]) out.t[7][o] = 4.0 * nu * val;
        break;
    case M_FX:
        if (out.t[1]) out.t[1][o] = PR(P_TX, j2) - PR(P_TX, j1) + val;
        break;
    case M_FY:
        if (out.t[4]) out.t[4][o] = PR(P_TY, j2) - PR(P_TY, j1) + val;
        break;
    case M_FZ:
        if (out.t[6]) out.t[6][o] = PR(P_TZ, j2) - PR(P_TZ, j1) + val;
        break;
    case M_PHI:
        if (out.t[8]) out.t[8][o] = 0.5 * (PR(P_TY, j1) + PR(P_TY, j2) + val);
        break;
    case M_PP:
        if (out.t[9]) out.t[9][o] = 2.0 * (PR(P_PV, j1) + PR(P_PV, j2) - val);
        break;
    case M_UVS:
        if (out.t[11])
            out.t[11][o] = -2.0 * (PR(P_UV, j1) + PR(P_UV, j2) - val) * 0.5 * (PR(P_S, j1) + PR(P_S, j2));
        break;
    default:  // M_UVA
        if (out.t[12]) out.t[12][o] = -(PR(P_UV, j2) - PR(P_UV, j1) + val) * (PR(P_S, j2) - PR(P_S, j1));
        break;
    }
#undef PR
}

// Inverse real transform along kx of 2*nt pairs (two real maps per complex
// transform), then assembly for pair (Y1, Y2) and, when the pair table asks
// for it, the mirrored pair (Y2, Y1) from r -> -r.
__global__ __launch_bounds__(256) void k_fin_kx(const cx<double> *__restrict__ mid, Dims d,
                                                Tables t, int p0, int ptot, int nt,
                                                const double *__restrict__ prof, OutPtrs out)
{
    extern __shared__ cx<double> lds[];
    const int nx = d.nx, nz = d.nz, nkx = d.nkx, ny = d.ny;
    const int npair = 2 * nt;
    const int pblk = blockIdx.x, rz = blockIdx.y, m = blockIdx.z;
    const int pl0 = pblk * npair;
    const int np = min(npair, ptot - pl0);
    const int bs = nx + 1;
    const int bsz = max(nt * bs, nkx * npair);
    cx<double> *A = lds;
    cx<double> *S = lds + nt * bs;   // staging, then FFT scratch
    for (int e = threadIdx.x; e < nkx * npair; e += blockDim.x) {
        const int kx = e / npair, b = e - kx * npair;
        S[kx * npair + b] = (b < np) ? mid[(((size_t)m * nkx + kx) * nz + rz) * ptot + pl0 + b]
                                     : cx<double>{0.0, 0.0};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * nx; e += blockDim.x) {
        const int c = e / nx, n = e - c * nx;
        cx<double> xa, xb;
        if (n <= nx / 2) {
            xa = S[n * npair + 2 * c];
            xb = S[n * npair + 2 * c + 1];
        } else {
            xa = cconj(S[(nx - n) * npair + 2 * c]);
            xb = cconj(S[(nx - n) * npair + 2 * c + 1]);
        }
        A[c * bs + n] = cx<double>{xa.x - xb.y, xa.y + xb.x};  // xa + i xb
    }
    __syncthreads();
    const cx<double> *R = lds_fft<double>(A, S, nt, bs, t.px, t.twx, +1);
    (void)bsz;
    const double sig = map_sigma(m);
    const size_t plane = (size_t)nz * nkx;
    for (int e = threadIdx.x; e < np * nkx; e += blockDim.x) {
        const int b = e / nkx, rx = e - b * nkx;
        const int code = t.pairs[p0 + pl0 + b];
        const int j1 = pair_j1(code), j2 = pair_j2(code);
        const int c = b >> 1;
        const cx<double> zv = R[c * bs + rx];
        const double val = (b & 1) ? zv.y : zv.x;
        assemble_store(m, val, j1, j2, prof, ny, d.nu, out,
                       ((size_t)j1 * ny + j2) * plane + (size_t)rz * nkx + rx);
        if (pair_mirror(code)) {
            const int rxm = (rx == 0) ? 0 : nx - rx;
            const cx<double> zm = R[c * bs + rxm];
            const double vm = sig * ((b & 1) ? zm.y : zm.x);
            const int rzm = (rz == 0) ? 0 : nz - rz;
            assemble_store(m, vm, j2, j1, prof, ny, d.nu, out,
                           ((size_t)j2 * ny + j1) * plane + (size_t)rzm * nkx + rx);
        }
    }
}

hipError_t launch_fin_kx(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *mid, int p0, int p1, const double *prof,
                         double *const *out)
{
    const int ptot = p1 - p0;
    int nt = 8;
    auto need = [&](int n) {
        return sizeof(cx<double>) * ((size_t)n * (d.nx + 1) +
                                     std::max((size_t)n * (d.nx + 1), (size_t)d.nkx * 2 * n));
    };
    while (nt > 1 && need(nt) > 65536) nt >>= 1;
    OutPtrs op;
    for (int i = 0; i < 14; ++i) op.t[i] = out[i];
    dim3 grid((ptot + 2 * nt - 1) / (2 * nt), d.nz, NMAP);
    hipLaunchKernelGGL(k_fin_kx, grid, dim3(256), need(nt), st, mid, d, t, p0, ptot, nt, prof, op);
    return hipGetLastError();
}

// Step 3: d/dY1 and d/dY2 of <du^2> with the five-point weights;
// T6 = -2 nu d/dry = -nu (d/dY2 - d/dY1), T11 = -(nu/2)(d/dY1 + d/dY2).
__global__ __launch_bounds__(256) void k_fd_terms(const double *__restrict__ t1, Dims d,
                                                  Tables t, double *__restrict__ t6,
                                                  double *__restrict__ t11)
{
    const int ny = d.ny;
    const size_t plane = (size_t)d.nz * d.nkx;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j2 = blockIdx.y, j1 = blockIdx.z;
    if (i >= plane) return;
    const int a1 = t.j0[j1], a2 = t.j0[j2];
    double d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        d1 += t.w5[j1 * 5 + a] * t1[((size_t)(a1 + a) * ny + j2) * plane + i];
        d2 += t.w5[j2 * 5 + a] * t1[((size_t)j1 * ny + a2 + a) * plane + i];
    }
    const size_t o = ((size_t)j1 * ny + j2) * plane + i;
    if (t6) t6[o] = -d.nu * (d2 - d1);
    if (t11) t11[o] = -0.5 * d.nu * (d1 + d2);
}

hipError_t launch_fd_terms(hipStream_t st, const Dims &d, const Tables &t, const double *t1,
                           double *t6, double *t11)
{
    const size_t plane = (size_t)d.nz * d.nkx;
    dim3 grid((unsigned)((plane + 255) / 256), d.ny, d.ny);
    hipLaunchKernelGGL(k_fd_terms, grid, dim3(256), 0, st, t1, d, t, t6, t11);
    return hipGetLastError();
}

}  // namespace gke
