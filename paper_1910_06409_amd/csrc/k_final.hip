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

template <typename F>
static void set_lds_limit(F *kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)LDS_BUDGET);
}

// Inverse transform along kz for pb pairs of one term spectrum at one kx.
// mid layout: [NMAP][nkx][nz (rz)][ptot (pairs of this batch)].
__global__ GKE_FFT_BOUNDS void k_fin_kz(const cx<double> *__restrict__ acc, Dims d,
                                                      Tables t, int p0, int ptot,
                                                      double inv_count,
                                                      cx<double> *__restrict__ mid)
{
    extern __shared__ cx<double> lds[];
    const int nz = d.nz, nkx = d.nkx, pb = d.pbz;
    const int pblk = blockIdx.x, kx = blockIdx.y, sp = blockIdx.z;
    const int pl0 = pblk * pb;                       // first pair within the batch
    const int np = min(pb, ptot - pl0);
    const size_t pall = (size_t)d.npair;
    const size_t pg0 = (size_t)p0 + pl0;             // first pair within acc
    const int bs = fft_stride(nz);
    const double two_pi = 6.283185307179586476925286766559;
    const double alpha = (2 * kx == d.nx) ? 0.0 : two_pi * kx / d.lx;
    const int nout_tr = (sp == S_R) ? 2 : 1;
    cx<double> *tw = lds + pb * bs;
    load_twiddles(tw, t.twz, nz);
    const cx<double> *ab = acc + ((size_t)sp * d.nk + (size_t)kx * nz) * pall + pg0;
    const int cnt = nz * np;
    for (int tr = 0; tr < nout_tr; ++tr) {
        // e = kz np + b: pairs contiguous in acc
        gather_batched<GKE_GATHER, FFT_BLOCK, cx<double>>(
            cnt,
            [&](int e) {
                const int kz = e / np, b = e - kz * np;
                return ab[kz * pall + b];
            },
            [&](int e, cx<double> X) {
                const int kz = e / np, b = e - kz * np;
                X = cscale(X, inv_count);
                if (tr == 1) {  // i beta R^
                    const int kzs = (kz <= nz / 2) ? kz : kz - nz;
                    const double beta = (2 * kz == nz) ? 0.0 : two_pi * kzs / d.lz;
                    X = cx<double>{-beta * X.y, beta * X.x};
                }
                lds[b * bs + fft_pad(kz)] = X;
            });
        __syncthreads();
        lds_fft_ip<double, FFT_CAP, FFT_BLOCK>(lds, np, bs, t.pz, tw, +1);
        int m0;
        if (sp == S_R) m0 = (tr == 0) ? M_R : M_DRZ;
        else m0 = M_FX + (sp - S_FX);  // FX FY FZ PHI PP UVS UVA map one to one
        Walk2 ws(threadIdx.x, FFT_BLOCK, np);   // (rz, b)
        for (int e = threadIdx.x; e < cnt; e += FFT_BLOCK) {
            const int rz = ws.hi, b = ws.lo;
            ws.next();
            const cx<double> Y = lds[b * bs + fft_pad(rz)];
            const size_t o = ((size_t)kx * nz + rz) * ptot + pl0 + b;
            mid[(size_t)m0 * nkx * nz * ptot + o] = Y;
            if (sp == S_R && tr == 0)  // i alpha R^: alpha is constant along kz
                mid[(size_t)M_DRX * nkx * nz * ptot + o] = cx<double>{-alpha * Y.y, alpha * Y.x};
        }
        __syncthreads();
    }
}

hipError_t launch_fin_kz(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *acc, int p0, int p1, double inv_count,
                         cx<double> *mid)
{
    const int ptot = p1 - p0;
    const size_t lds = sizeof(cx<double>) * ((size_t)d.pbz * fft_stride(d.nz) + d.nz);
    dim3 grid((ptot + d.pbz - 1) / d.pbz, d.nkx, NSPEC);
    set_lds_limit(k_fin_kz);
    hipLaunchKernelGGL(k_fin_kz, grid, dim3(FFT_BLOCK), lds, st, acc, d, t, p0, ptot, inv_count,
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
__global__ GKE_FFT_BOUNDS void k_fin_kx(const cx<double> *__restrict__ mid, Dims d,
                                                      Tables t, int p0, int ptot,
                                                      const double *__restrict__ prof,
                                                      OutPtrs out, int full)
{
    extern __shared__ cx<double> lds[];
    const int nx = d.nx, nz = d.nz, nkx = d.nkx, ny = d.ny, nt = d.ntx;
    const int npair = 2 * nt;
    const int pblk = blockIdx.x, rz = blockIdx.y, m = blockIdx.z;
    const int pl0 = pblk * npair;
    const int np = min(npair, ptot - pl0);
    const int bs = fft_stride(nx);
    cx<double> *A = lds;                      // nt transforms of length nx
    cx<double> *S = lds + nt * bs;            // staging [kx][pair]
    cx<double> *tw = S + nkx * npair;         // twiddles
    load_twiddles(tw, t.twx, nx);
    {
        // e = kx npair + b: the pairs of one (map, kx, rz) are contiguous in mid
        const cx<double> *mb = mid + ((size_t)m * nkx * nz + rz) * ptot + pl0;
        const size_t skx = (size_t)nz * ptot;
        const int cnt = nkx * npair;
        for (int base = 0; base < cnt; base += GKE_GATHER * FFT_BLOCK) {
            Walk2 w(base + threadIdx.x, FFT_BLOCK, npair);   // (kx, b)
            cx<double> v[GKE_GATHER];
#pragma unroll
            for (int q = 0; q < GKE_GATHER; ++q) {
                v[q] = cx<double>{0.0, 0.0};
                if (base + (int)threadIdx.x + q * FFT_BLOCK < cnt && w.lo < np)
                    v[q] = mb[w.hi * skx + w.lo];
                w.next();
            }
#pragma unroll
            for (int q = 0; q < GKE_GATHER; ++q) {
                const int e = base + threadIdx.x + q * FFT_BLOCK;
                if (e < cnt) S[e] = v[q];
            }
        }
    }
    __syncthreads();
    // consecutive threads take consecutive transforms: bank-friendly reads of S
    Walk2 wn(threadIdx.x, FFT_BLOCK, nt);   // (n, c)
    for (int e = threadIdx.x; e < nt * nx; e += FFT_BLOCK) {
        const int n = wn.hi, c = wn.lo;
        wn.next();
        cx<double> xa, xb;
        if (n <= nx / 2) {
            xa = S[n * npair + 2 * c];
            xb = S[n * npair + 2 * c + 1];
        } else {
            xa = cconj(S[(nx - n) * npair + 2 * c]);
            xb = cconj(S[(nx - n) * npair + 2 * c + 1]);
        }
        A[c * bs + fft_pad(n)] = cx<double>{xa.x - xb.y, xa.y + xb.x};  // xa + i xb
    }
    __syncthreads();
    lds_fft_ip<double, FFT_CAP, FFT_BLOCK>(A, nt, bs, t.px, tw, +1);
    if (full) {
        // one orientation, every rx, rows of the full-plane buffer
        Walk2 wb(threadIdx.x, FFT_BLOCK, nx);   // (b, rx)
        for (int e = threadIdx.x; e < np * nx; e += FFT_BLOCK) {
            const int b = wb.hi, rx = wb.lo;
            wb.next();
            const int code = t.pairs[p0 + pl0 + b];
            const int j1 = pair_j1(code), j2 = pair_j2(code);
            const cx<double> zv = A[(b >> 1) * bs + fft_pad(rx)];
            const double val = (b & 1) ? zv.y : zv.x;
            assemble_store(m, val, j1, j2, prof, ny, d.nu, out,
                           (((size_t)t.rowidx[j1] * ny + j2) * nz + rz) * nx + rx);
        }
        return;
    }
    const double sig = map_sigma(m);
    const size_t plane = (size_t)nz * nkx;
    Walk2 wb(threadIdx.x, FFT_BLOCK, nkx);   // (b, rx)
    for (int e = threadIdx.x; e < np * nkx; e += FFT_BLOCK) {
        const int b = wb.hi, rx = wb.lo;
        wb.next();
        const int code = t.pairs[p0 + pl0 + b];
        const int j1 = pair_j1(code), j2 = pair_j2(code);
        const int c = b >> 1;
        const cx<double> zv = A[c * bs + fft_pad(rx)];
        const double val = (b & 1) ? zv.y : zv.x;
        assemble_store(m, val, j1, j2, prof, ny, d.nu, out,
                       ((size_t)j1 * ny + j2) * plane + (size_t)rz * nkx + rx);
        if (pair_mirror(code)) {
            const int rxm = (rx == 0) ? 0 : nx - rx;
            const cx<double> zm = A[c * bs + fft_pad(rxm)];
            const double vm = sig * ((b & 1) ? zm.y : zm.x);
            const int rzm = (rz == 0) ? 0 : nz - rz;
            assemble_store(m, vm, j2, j1, prof, ny, d.nu, out,
                           ((size_t)j2 * ny + j1) * plane + (size_t)rzm * nkx + rx);
        }
    }
}

hipError_t launch_fin_kx(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *mid, int p0, int p1, const double *prof,
                         double *const *out, int full)
{
    const int ptot = p1 - p0;
    const size_t lds = sizeof(cx<double>) *
                       ((size_t)d.ntx * fft_stride(d.nx) + (size_t)d.nkx * 2 * d.ntx + d.nx);
    OutPtrs op;
    for (int i = 0; i < 14; ++i) op.t[i] = out[i];
    dim3 grid((ptot + 2 * d.ntx - 1) / (2 * d.ntx), d.nz, NMAP);
    set_lds_limit(k_fin_kx);
    hipLaunchKernelGGL(k_fin_kx, grid, dim3(FFT_BLOCK), lds, st, mid, d, t, p0, ptot, prof, op,
                       full);
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

// Output of one slab in the general modes.  The maps of the slab's rows, of
// their five-point neighbours and (with the mirror average) of the reflected
// rows sit in the full-plane buffer mf[slot][row][Y2][rz][rx < Nx] for the
// eleven terms that come from the transforms (slot k of term t: kslot below).
// For every output pair (Y1, Y2) of the slab (opairs[q] = Y1 | Y2 << 16) and
// every (rz, rx < width):
//   mirror = 1: the average with the reflected pair,
//     (T(Y1, Y2) + sigma_y T(2h - Y1, 2h - Y2)) / 2   (Section "Step 2": the
//     other half of the channel doubles the sample; sigma_y = sign of the term
//     under the reflection, Section "Exploiting symmetries");
//   T6, T11 from the five-point Y1 and Y2 derivatives of the (averaged) <du^2>
//   (Section "Step 3"), T14 from eps.
// out[t][(q Nz + rz) width + rx]; T14 out[13][q].
struct OutPtrs14 {
    double *t[14];
};

__global__ __launch_bounds__(256) void k_slab_out(const double *__restrict__ mf, size_t mstride,
                                                  Dims d, Tables t,
                                                  const int *__restrict__ opairs,
                                                  const double *__restrict__ prof, int mirror,
                                                  int width, OutPtrs14 out)
{
    // slot of each term in mf (-1: not a transformed map)
    constexpr int kslot[14] = {0, 1, 2, 3, 4, -1, 5, 6, 7, 8, -1, 9, 10, -1};
    constexpr double sig[14] = {1, 1, 1, 1, -1, -1, 1, 1, -1, -1, -1, 1, 1, 1};
    const int ny = d.ny, nz = d.nz, nx = d.nx;
    const int q = blockIdx.x, rz = blockIdx.y;
    const int code = opairs[q];
    const int j1 = code & 0xffff, j2 = code >> 16;
    const size_t plane = (size_t)nz * nx;
    auto M = [&](int slot, int r, int c, size_t ofs) {
        return mf[slot * mstride + ((size_t)t.rowidx[r] * ny + c) * plane + ofs];
    };
    auto Tb = [&](int slot, int r, int c, size_t ofs, double sg) {
        double v = M(slot, r, c, ofs);
        if (mirror) v = 0.5 * (v + sg * M(slot, ny - 1 - r, ny - 1 - c, ofs));
        return v;
    };
    const bool fd = out.t[5] || out.t[10];
    const int a1 = t.j0[j1], a2 = t.j0[j2];
    for (int rx = threadIdx.x; rx < width; rx += blockDim.x) {
        const size_t ofs = (size_t)rz * nx + rx;
        const size_t o = ((size_t)q * nz + rz) * width + rx;
#pragma unroll
        for (int k = 0; k < 14; ++k)
            if (kslot[k] >= 0 && out.t[k]) out.t[k][o] = Tb(kslot[k], j1, j2, ofs, sig[k]);
        if (fd) {
            double d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                d1 += t.w5[j1 * 5 + a] * Tb(0, a1 + a, j2, ofs, 1.0);
                d2 += t.w5[j2 * 5 + a] * Tb(0, j1, a2 + a, ofs, 1.0);
            }
            if (out.t[5]) out.t[5][o] = -d.nu * (d2 - d1);
            if (out.t[10]) out.t[10][o] = -0.5 * d.nu * (d1 + d2);
        }
    }
    if (out.t[13] && rz == 0 && threadIdx.x == 0) {
        const double *eps = prof + P_EPS * ny;
        double v = -2.0 * (eps[j1] + eps[j2]);
        if (mirror) v = 0.5 * (v - 2.0 * (eps[ny - 1 - j1] + eps[ny - 1 - j2]));
        out.t[13][q] = v;
    }
}

hipError_t launch_slab_out(hipStream_t st, const Dims &d, const Tables &t, const double *mf,
                           size_t mstride, const int *opairs, int nopairs, const double *prof,
                           int mirror, int width, double *const *out)
{
    OutPtrs14 op;
    for (int i = 0; i < 14; ++i) op.t[i] = out[i];
    if (nopairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slab_out, dim3(nopairs, d.nz), dim3(256), 0, st, mf, mstride, d, t,
                       opairs, prof, mirror, width, op);
    return hipGetLastError();
}

}  // namespace gke
