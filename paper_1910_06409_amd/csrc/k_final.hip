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

__host__ __device__ inline int mid_stride(int ptot) { return (ptot + 7) & ~7; }

// Inverse transform along kz of the pairs of one term spectrum at one kx.
// Blocks z = 0, 1 take the two halves of a block of pb pairs of the R spectrum
// and transform R^ and i beta R^ together (2 * pb/2 transforms); blocks z >= 2
// take pb pairs of spectrum z - 1.  Every block reads its part of acc once.
// mid layout: [NMID][nkx][nz (rz)][mid_stride(ptot)] (the pairs of this batch,
// rows padded to whole 128-byte lines).
template <int NF>
__global__ GKE_FFT_BOUNDS void k_fin_kz(const cx<double> *__restrict__ acc, Dims d,
                                                      Tables t, int p0, int ptot,
                                                      double inv_count,
                                                      cx<double> *__restrict__ mid)
{
    extern __shared__ cx<double> lds[];
    // NF > 0: the z length as a constant (its plan compiled in)
    const int nz = NF > 0 ? NF : d.nz, nkx = d.nkx, pb = d.pbz;   // pb even (host)
    const int kx = blockIdx.y;
    const bool isr = blockIdx.z < 2;
    const int sp = isr ? (int)S_R : (int)blockIdx.z - 1;
    const int pl0 = blockIdx.x * pb + (isr ? (int)blockIdx.z * (pb >> 1) : 0);
    const int np = min(isr ? pb >> 1 : pb, ptot - pl0);   // pairs of this block
    if (np <= 0) return;                                   // whole block
    const size_t pall = (size_t)d.pstr;
    const size_t mst = (size_t)mid_stride(ptot);
    const int bs = fft_stride(nz);
    const double two_pi = 6.283185307179586476925286766559;
    cx<double> *tw = lds + pb * bs;
    const cx<double> *ab = acc + ((size_t)sp * d.nk + (size_t)kx * nz) * pall + p0 + pl0;
    const int cnt = nz * np;
    {
        // nz * np <= FFT_CAP: every load of this thread is in flight at once.
        // Loads and LDS stores are unconditional (no branch holds a load and
        // its wait): a slot past the end takes element (nz - 1, 0) and stores
        // it where that element goes.  e = kz np + b (pairs contiguous in acc),
        // walked without divisions.
        constexpr int MAXE = (FFT_CAP + FFT_BLOCK - 1) / FFT_BLOCK;
        cx<double> x[MAXE];
        const int ps = (int)pall;   // nz * pall < 2^31 (host)
        Walk2 w(threadIdx.x, FFT_BLOCK, np);   // (kz, b)
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nz;
            x[q] = ab[(ok ? w.hi : nz - 1) * ps + (ok ? w.lo : 0)];
            w.next();
        }
        TwiddleCopy<double, FFT_BLOCK> twc;   // in flight with the gathers
        twc.load(t.twz, nz);
        twc.store(tw, t.twz, nz);
        w = Walk2(threadIdx.x, FFT_BLOCK, np);
        const double bscale = two_pi / d.lz;
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nz;
            const int kz = ok ? w.hi : nz - 1, b = ok ? w.lo : 0;
            w.next();
            const cx<double> X = cscale(x[q], inv_count);
            lds[b * bs + fft_pad(kz)] = X;
            if (isr) {   // i beta R^ as transform np + b
                const int kzs = (kz <= nz / 2) ? kz : kz - nz;
                const double beta = (2 * kz == nz) ? 0.0 : bscale * kzs;
                lds[(np + b) * bs + fft_pad(kz)] = cx<double>{-beta * X.y, beta * X.x};
            }
        }
    }
    __syncthreads();
    lds_fft<double, NF, FFT_CAP, FFT_BLOCK, +1>(lds, isr ? 2 * np : np, bs, t.pz, tw);
    const size_t mplane = (size_t)nkx * nz * mst;
    Walk2 ws(threadIdx.x, FFT_BLOCK, np);   // (rz, b)
    for (int e = threadIdx.x; e < cnt; e += FFT_BLOCK) {
        const int rz = ws.hi, b = ws.lo;
        ws.next();
        const cx<double> Y = lds[b * bs + fft_pad(rz)];
        const size_t o = ((size_t)kx * nz + rz) * mst + pl0 + b;
        if (isr) {
            mid[(size_t)mid_plane(M_R) * mplane + o] = Y;
            mid[(size_t)mid_plane(M_DRZ) * mplane + o] = lds[(np + b) * bs + fft_pad(rz)];
        } else {
            mid[(size_t)mid_plane(M_FX + (sp - S_FX)) * mplane + o] = Y;   // FX .. UVA one to one
        }
    }
}

hipError_t launch_fin_kz(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *acc, int p0, int p1, double inv_count,
                         cx<double> *mid)
{
    const int ptot = p1 - p0;
    const size_t lds = sizeof(cx<double>) * ((size_t)d.pbz * fft_stride(d.nz) + d.nz);
    dim3 grid((ptot + d.pbz - 1) / d.pbz, d.nkx, NSPEC + 1);
    with_fft_len(d.nz, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        set_lds_limit(k_fin_kz<NF>);
        hipLaunchKernelGGL(k_fin_kz<NF>, grid, dim3(FFT_BLOCK), lds, st, acc, d, t, p0, ptot,
                           inv_count, mid);
    });
    return hipGetLastError();
}

// Residual of the budget, homogeneous part (eq. GKE-conservative: the r_x and
// r_z divergence of the scale fluxes, spectral as in Section "GKE and
// turbulence physics").  With Phi_rx = T2 + T3 + T4 and Phi_rz = T7 + T8, whose
// r-dependent spectra are FX^ (T2), -2 dU R^ (T3 = dU <du^2>, <du^2> = const
// - 2 R), 4 nu i alpha R^ (T4), FZ^ (T7) and 4 nu i beta R^ (T8):
//   H^ = i alpha FX^ + i beta FZ^ - 2 dU i alpha R^ - 4 nu (alpha^2 + beta^2) R^,
// dU = U(Y2) - U(Y1), zero multipliers at the Nyquist wavenumbers.  One block
// per (pb pairs, kx): the three spectra are read one after the other into the
// same per-thread elements, then the kz transform as in k_fin_kz, into mid
// plane NMID.
constexpr int MAX_PBZ = 16;
template <int NF>
__global__ GKE_FFT_BOUNDS void k_fin_kz_h(const cx<double> *__restrict__ acc, Dims d, Tables t,
                                          int p0, int ptot, double inv_count,
                                          const double *__restrict__ prof,
                                          cx<double> *__restrict__ mid)
{
    extern __shared__ cx<double> lds[];
    __shared__ double sdu[MAX_PBZ];
    const int nz = NF > 0 ? NF : d.nz, nkx = d.nkx, pb = d.pbz, ny = d.ny;   // pb <= MAX_PBZ (host)
    const int kx = blockIdx.y;
    const int pl0 = blockIdx.x * pb;
    const int np = min(pb, ptot - pl0);
    if (np <= 0) return;                                       // whole block
    const size_t pall = (size_t)d.pstr;
    const size_t mst = (size_t)mid_stride(ptot);
    const int bs = fft_stride(nz);
    const double two_pi = 6.283185307179586476925286766559;
    cx<double> *tw = lds + pb * bs;
    if ((int)threadIdx.x < np) {
        const int code = t.pairs[p0 + pl0 + threadIdx.x];
        sdu[threadIdx.x] = prof[P_U * ny + pair_j2(code)] - prof[P_U * ny + pair_j1(code)];
    }
    TwiddleCopy<double, FFT_BLOCK> twc;
    twc.load(t.twz, nz);
    twc.store(tw, t.twz, nz);
    __syncthreads();
    const double al = (2 * kx == d.nx) ? 0.0 : two_pi * kx / d.lx;
    const double bscale = two_pi / d.lz;
    const int ps = (int)pall;   // nz * pall < 2^31 (host)
    constexpr int MAXE = (FFT_CAP + FFT_BLOCK - 1) / FFT_BLOCK;
    cx<double> h[MAXE];
    // elements past the end take (nz - 1, 0) and compute its value (stores repeat it)
    const int sps[3] = {S_R, S_FX, S_FZ};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const cx<double> *ab = acc + ((size_t)sps[k] * d.nk + (size_t)kx * nz) * pall + p0 + pl0;
        cx<double> x[MAXE];
        Walk2 w(threadIdx.x, FFT_BLOCK, np);   // (kz, b)
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nz;
            x[q] = ab[(ok ? w.hi : nz - 1) * ps + (ok ? w.lo : 0)];
            w.next();
        }
        w = Walk2(threadIdx.x, FFT_BLOCK, np);
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nz;
            const int kz = ok ? w.hi : nz - 1, b = ok ? w.lo : 0;
            w.next();
            const int kzs = (kz <= nz / 2) ? kz : kz - nz;
            const double be = (2 * kz == nz) ? 0.0 : bscale * kzs;
            const cx<double> X = cscale(x[q], inv_count);
            if (k == 0) {        // -(2 dU i alpha + 4 nu (alpha^2 + beta^2)) R^
                const double c = -4.0 * d.nu * (al * al + be * be), s = -2.0 * sdu[b] * al;
                h[q] = cx<double>{c * X.x - s * X.y, c * X.y + s * X.x};
            } else if (k == 1) { // + i alpha FX^
                h[q] = cx<double>{h[q].x - al * X.y, h[q].y + al * X.x};
            } else {             // + i beta FZ^
                h[q] = cx<double>{h[q].x - be * X.y, h[q].y + be * X.x};
                lds[b * bs + fft_pad(kz)] = h[q];
            }
        }
    }
    __syncthreads();
    lds_fft<double, NF, FFT_CAP, FFT_BLOCK, +1>(lds, np, bs, t.pz, tw);
    const size_t mplane = (size_t)nkx * nz * mst;
    const int cnt = nz * np;
    Walk2 ws(threadIdx.x, FFT_BLOCK, np);   // (rz, b)
    for (int e = threadIdx.x; e < cnt; e += FFT_BLOCK) {
        const int rz = ws.hi, b = ws.lo;
        ws.next();
        mid[(size_t)NMID * mplane + ((size_t)kx * nz + rz) * mst + pl0 + b] =
            lds[b * bs + fft_pad(rz)];
    }
}

hipError_t launch_fin_kz_h(hipStream_t st, const Dims &d, const Tables &t,
                           const cx<double> *acc, int p0, int p1, double inv_count,
                           const double *prof, cx<double> *mid)
{
    if (d.pbz > MAX_PBZ) return hipErrorInvalidValue;
    const int ptot = p1 - p0;
    const size_t lds = sizeof(cx<double>) * ((size_t)d.pbz * fft_stride(d.nz) + d.nz);
    dim3 grid((ptot + d.pbz - 1) / d.pbz, d.nkx, 1);
    with_fft_len(d.nz, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        set_lds_limit(k_fin_kz_h<NF>);
        hipLaunchKernelGGL(k_fin_kz_h<NF>, grid, dim3(FFT_BLOCK), lds, st, acc, d, t, p0, ptot,
                           inv_count, prof, mid);
    });
    return hipGetLastError();
}

// Output maps are FP64 or FP32 (f32 = 1: every value, assembled in FP64, is
// rounded once when stored); the flag is uniform over a launch.
__device__ __forceinline__ void put(void *p, size_t o, double v, int f32)
{
    if (f32) static_cast<float *>(p)[o] = (float)v;
    else static_cast<double *>(p)[o] = v;
}
__device__ __forceinline__ double get(const void *p, size_t o, int f32)
{
    return f32 ? (double)static_cast<const float *>(p)[o] : static_cast<const double *>(p)[o];
}

struct OutPtrs {
    void *t[14];
    void *res;     // residual map (its homogeneous part, map M_H), or NULL
    int f32;       // maps stored as FP32
};

// sign of each map under r-inversion: map(r; Y2, Y1) = sigma * map(-r; Y1, Y2)
__device__ __forceinline__ double map_sigma(int m)
{
    switch (m) {
    case M_R: case M_PHI: case M_PP: case M_UVS: case M_H: return 1.0;
    default: return -1.0;
    }
}

// One-point profile rows that map m combines with: a (and b) at Y1 and Y2.
__device__ __forceinline__ void map_rows(int m, int &ra, int &rb)
{
    rb = -1;
    switch (m) {
    case M_R: ra = P_Q; rb = P_U; break;
    case M_FX: ra = P_TX; break;
    case M_FY: case M_PHI: ra = P_TY; break;
    case M_FZ: ra = P_TZ; break;
    case M_PP: ra = P_PV; break;
    case M_UVS: case M_UVA: ra = P_UV; rb = P_S; break;
    default: ra = -1; break;   // M_DRX, M_DRZ
    }
}

// Assemble the terms that use map m and store them at index o; a1 a2 (b1 b2)
// are the profile rows of map_rows at the first and the second plane.
__device__ __forceinline__ void assemble_store(int m, double val, double a1, double a2,
                                               double b1, double b2, double nu,
                                               const OutPtrs &out, size_t o)
{
    const int f = out.f32;
    switch (m) {
    case M_R: {
        const double t1 = a1 + a2 - 2.0 * val;                // <du^2>
        if (out.t[0]) put(out.t[0], o, t1, f);
        if (out.t[2]) put(out.t[2], o, (b2 - b1) * t1, f);     // <du^2 dU>
        break;
    }
    case M_DRX:
        if (out.t[3]) put(out.t[3], o, 4.0 * nu * val, f);
        break;
    case M_DRZ:
        if (out.t[7]) put(out.t[7], o, 4.0 * nu * val, f);
        break;
    case M_FX:
        if (out.t[1]) put(out.t[1], o, a2 - a1 + val, f);
        break;
    case M_FY:
        if (out.t[4]) put(out.t[4], o, a2 - a1 + val, f);
        break;
    case M_FZ:
        if (out.t[6]) put(out.t[6], o, a2 - a1 + val, f);
        break;
    case M_PHI:
        if (out.t[8]) put(out.t[8], o, 0.5 * (a1 + a2 + val), f);
        break;
    case M_PP:
        if (out.t[9]) put(out.t[9], o, 2.0 * (a1 + a2 - val), f);
        break;
    case M_UVS:
        if (out.t[11]) put(out.t[11], o, -2.0 * (a1 + a2 - val) * 0.5 * (b1 + b2), f);
        break;
    case M_H:
        if (out.res) put(out.res, o, val, f);
        break;
    default:  // M_UVA
        if (out.t[12]) put(out.t[12], o, -(a2 - a1 + val) * (b2 - b1), f);
        break;
    }
}

// per-pair data of a kx block, staged in LDS before the transform
struct PairInfo {
    int j1, j2, mirror, row1;   // row1: output row of j1 in the full-plane mode
    double a1, a2, b1, b2;
};

// Inverse real transform along kx of 2*nt pairs (two real maps per complex
// transform), then assembly for pair (Y1, Y2) and, when the pair table asks
// for it, the mirrored pair (Y2, Y1) from r -> -r.
//   Transform c packs pairs 2c and 2c + 1: A_c[n] = X_2c[n] + i X_2c+1[n] with
//   X[n] for n > Nx/2 from Hermitian symmetry, X[Nx - kx] = conj X[kx], and
//   the real parts of X[0] and X[Nx/2] (values of real maps); the real and
//   imaginary parts of its inverse are the two maps.  A thread loads both
//   pairs of (kx, c) (adjacent in mid) and writes A_c[kx] and A_c[Nx - kx].
//   Output: a group of tpp consecutive threads per pair, consecutive threads
//   on consecutive rx.
template <int BLOCK, int NF>
__global__ __launch_bounds__(BLOCK, GKE_FFT_WAVES) void k_fin_kx(const cx<double> *__restrict__ mid, Dims d,
                                                      Tables t, int p0, int ptot,
                                                      const double *__restrict__ prof,
                                                      OutPtrs out, int full)
{
    constexpr int CAP = cap_of<BLOCK>();
    extern __shared__ cx<double> lds[];
    // NF > 0: the x length as a constant (its plan compiled in)
    const int nx = NF > 0 ? NF : d.nx, nz = d.nz, nkx = nx / 2 + 1, ny = d.ny, nt = d.ntx;
    const int npair = 2 * nt;
    const int pblk = blockIdx.x, m = blockIdx.z;
    // full-plane mode: every rz; all-pairs mode: the kept rz rows only
    const int rz = full ? (int)blockIdx.y : t.rzk[blockIdx.y];
    const int pl0 = pblk * npair;
    const int np = min(npair, ptot - pl0);
    const int bs = fft_stride(nx);
    cx<double> *A = lds;            // nt transforms of length nx
    cx<double> *tw = lds + nt * bs;   // twiddles
    __shared__ PairInfo pinfo[2 * MAX_NTX];
    // Every global load is issued before the first LDS store, so that the
    // block waits about two round trips (pair code, then everything else).
    // Loads and stores are unconditional at clamped indices (no branch holds
    // a load and its wait): a slot past the end repeats the last element,
    // which writes the same values to the same place.
    const int code = t.pairs[p0 + pl0 + min((int)threadIdx.x, np - 1)];
    // nkx * nt <= CAP / 2 + MAX_NTX (nt * fft_stride(nx) <= CAP, host)
    constexpr int MAXG = (CAP / 2 + MAX_NTX + BLOCK - 1) / BLOCK;
    const int cnt = nkx * nt;
    cx<double> xa[MAXG], xb[MAXG];
    const size_t mst = (size_t)mid_stride(ptot);
    {
        const cx<double> *mb = mid + ((size_t)mid_plane(m) * nkx * nz + rz) * mst + pl0;
        const size_t skx = (size_t)nz * mst;
        Walk2 w(threadIdx.x, BLOCK, nt);   // (kx, c)
#pragma unroll
        for (int q = 0; q < MAXG; ++q) {
            const bool ok = w.hi < nkx;
            const cx<double> *src = mb + (ok ? w.hi : nkx - 1) * skx;
            const int c = ok ? w.lo : nt - 1;
            xa[q] = src[min(2 * c, np - 1)];
            xb[q] = src[min(2 * c + 1, np - 1)];
            w.next();
        }
    }
    PairInfo pi;
    pi.j1 = pair_j1(code);
    pi.j2 = pair_j2(code);
    pi.mirror = pair_mirror(code);
    pi.row1 = full ? t.rowidx[pi.j1] : 0;
    {
        int ra, rb;
        map_rows(m, ra, rb);
        pi.a1 = ra >= 0 ? prof[ra * ny + pi.j1] : 0.0;
        pi.a2 = ra >= 0 ? prof[ra * ny + pi.j2] : 0.0;
        pi.b1 = rb >= 0 ? prof[rb * ny + pi.j1] : 0.0;
        pi.b2 = rb >= 0 ? prof[rb * ny + pi.j2] : 0.0;
    }
    {
        TwiddleCopy<double, BLOCK> twc;
        twc.load(t.twx, nx);
        twc.store(tw, t.twx, nx);
    }
    {
        Walk2 w(threadIdx.x, BLOCK, nt);   // (kx, c)
#pragma unroll
        for (int q = 0; q < MAXG; ++q) {
            const bool ok = w.hi < nkx;
            const int kx = ok ? w.hi : nkx - 1, c = ok ? w.lo : nt - 1;
            w.next();
            const cx<double> zero = cx<double>{0.0, 0.0};
            cx<double> a = 2 * c < np ? xa[q] : zero;      // padding pairs read 0
            cx<double> b = 2 * c + 1 < np ? xb[q] : zero;
            if (m == M_DRX) {   // i alpha R^, read from the R plane (0 at the Nyquist kx)
                const double al = (2 * kx == nx) ? 0.0 : 6.283185307179586476925286766559 * kx / d.lx;
                a = cx<double>{-al * a.y, al * a.x};
                b = cx<double>{-al * b.y, al * b.x};
            }
            cx<double> *Ac = A + c * bs;
            const bool self = kx == 0 || 2 * kx == nx;   // its own Hermitian partner
            if (self) {
                // the kz-transformed values of a real map at kx = 0 and Nx/2 are
                // real; keeping the real parts is the Hermitian average of the
                // accumulated +kz and -kz bins (exact for exact spectra), so
                // their rounding does not leak into the other pair of the
                // packed transform
                Ac[fft_pad(kx)] = cx<double>{a.x, b.x};
            } else {
                Ac[fft_pad(kx)] = cx<double>{a.x - b.y, a.y + b.x};          // a + i b
                Ac[fft_pad(nx - kx)] = cx<double>{a.x + b.y, b.x - a.y};     // conj a + i conj b
            }
        }
    }
    if ((int)threadIdx.x < np) pinfo[threadIdx.x] = pi;
    __syncthreads();
    lds_fft<double, NF, CAP, BLOCK, +1>(A, nt, bs, t.px, tw);
    const int tpp = BLOCK / npair;            // threads per pair
    const int b = threadIdx.x / tpp, lane = threadIdx.x - b * tpp;
    if (b >= np) return;
    const PairInfo p = pinfo[b];
    const cx<double> *Ac = A + (b >> 1) * bs;
    if (full) {
        // one orientation, every rx, rows of the full-plane buffer
        const size_t o0 = (((size_t)p.row1 * ny + p.j2) * nz + rz) * nx;
        for (int rx = lane; rx < nx; rx += tpp) {
            const cx<double> zv = Ac[fft_pad(rx)];
            assemble_store(m, (b & 1) ? zv.y : zv.x, p.a1, p.a2, p.b1, p.b2, d.nu, out, o0 + rx);
        }
        return;
    }
    // output maps [Y1][Y2][row of rz][column of rx] over the kept separations
    // (every rz and rx <= Nx/2 without undersampling: identity tables); the
    // kept set is symmetric in the sign of the separation, so -rz is kept too
    const double sig = map_sigma(m);
    const int npo = d.npo;
    const bool sampled = npo != nkx;
    const size_t plane = (size_t)d.nqo * npo;
    const size_t o0 = ((size_t)p.j1 * ny + p.j2) * plane + (size_t)blockIdx.y * npo;
    const int rzm = (rz == 0) ? 0 : nz - rz;
    const size_t om = ((size_t)p.j2 * ny + p.j1) * plane + (size_t)t.rzinv[rzm] * npo;
    for (int c = lane; c < npo; c += tpp) {
        const int rx = sampled ? t.rxk[c] : c;
        const cx<double> zv = Ac[fft_pad(rx)];
        assemble_store(m, (b & 1) ? zv.y : zv.x, p.a1, p.a2, p.b1, p.b2, d.nu, out, o0 + c);
        if (p.mirror) {   // (Y2, Y1) at -r: the profile roles swap
            const cx<double> zm = Ac[fft_pad(rx == 0 ? 0 : nx - rx)];
            const double vm = sig * ((b & 1) ? zm.y : zm.x);
            assemble_store(m, vm, p.a2, p.a1, p.b2, p.b1, d.nu, out, om + c);
        }
    }
}

hipError_t launch_fin_kx(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *mid, int p0, int p1, const double *prof,
                         void *const *out, int f32, int full, void *resid)
{
    const int ptot = p1 - p0;
    const size_t lds = sizeof(cx<double>) * ((size_t)d.ntx * fft_stride(d.nx) + d.nx);
    OutPtrs op;
    for (int i = 0; i < 14; ++i) op.t[i] = out[i];
    op.res = full ? nullptr : resid;
    op.f32 = f32;
    dim3 grid((ptot + 2 * d.ntx - 1) / (2 * d.ntx), full ? d.nz : d.nqo, NMAP + (op.res ? 1 : 0));
    with_fft_len(d.nx, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        if (d.kxblk == SMALL_BLOCK) {
            set_lds_limit(k_fin_kx<SMALL_BLOCK, NF>);
            hipLaunchKernelGGL((k_fin_kx<SMALL_BLOCK, NF>), grid, dim3(SMALL_BLOCK), lds, st, mid,
                               d, t, p0, ptot, prof, op, full);
        } else {
            set_lds_limit(k_fin_kx<FFT_BLOCK, NF>);
            hipLaunchKernelGGL((k_fin_kx<FFT_BLOCK, NF>), grid, dim3(FFT_BLOCK), lds, st, mid, d,
                               t, p0, ptot, prof, op, full);
        }
    });
    return hipGetLastError();
}

// Step 3: d/dY1 and d/dY2 of <du^2> with the five-point weights;
// T6 = -2 nu d/dry = -nu (d/dY2 - d/dY1), T11 = -(nu/2)(d/dY1 + d/dY2).
// Blocks in the order (tile of FD_TY rows Y1, Y2, row within the tile, chunk
// of the plane), chunk fastest; the blocks of one XCD (workgroup i runs on XCD
// i mod 8) take a contiguous range of that order.  A tile's blocks for one Y2
// read the tile's rows and their stencil halo once into L2, and the next Y2
// finds four of its five stencil columns there.
constexpr int FD_TY = 4;
__global__ __launch_bounds__(256) void k_fd_terms(const void *__restrict__ t1, Dims d,
                                                  Tables t, void *__restrict__ t6,
                                                  void *__restrict__ t11, int f32, int nchunk)
{
    const int ny = d.ny;
    const size_t plane = (size_t)d.nqo * d.npo;   // output map points per pair
    const int nb = (int)gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7;
    const int item = xcd * q8 + min(xcd, r8) + (int)(blockIdx.x >> 3);
    const int chunk = item % nchunk, r = item / nchunk;
    const int yi = r % FD_TY, j2 = (r / FD_TY) % ny, tile = r / (FD_TY * ny);
    const int j1 = tile * FD_TY + yi;
    const size_t i = (size_t)chunk * blockDim.x + threadIdx.x;
    if (j1 >= ny || i >= plane) return;
    const int a1 = t.j0[j1], a2 = t.j0[j2];
    double d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        d1 += t.w5[j1 * 5 + a] * get(t1, ((size_t)(a1 + a) * ny + j2) * plane + i, f32);
        d2 += t.w5[j2 * 5 + a] * get(t1, ((size_t)j1 * ny + a2 + a) * plane + i, f32);
    }
    const size_t o = ((size_t)j1 * ny + j2) * plane + i;
    if (t6) put(t6, o, -d.nu * (d2 - d1), f32);
    if (t11) put(t11, o, -0.5 * d.nu * (d1 + d2), f32);
}

hipError_t launch_fd_terms(hipStream_t st, const Dims &d, const Tables &t, const void *t1,
                           void *t6, void *t11, int f32)
{
    const size_t plane = (size_t)d.nqo * d.npo;   // output map points per pair
    const int nchunk = (int)((plane + 255) / 256);
    const size_t nblk = (size_t)nchunk * d.ny * ((d.ny + FD_TY - 1) / FD_TY) * FD_TY;
    if (nblk >= ((size_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fd_terms, dim3((unsigned)nblk), dim3(256), 0, st, t1, d, t, t6, t11,
                       f32, nchunk);
    return hipGetLastError();
}

// Residual, wall-normal part and sources (eq. GKE-conservative; Section
// "Step 3": d/dry = (d/dY2 - d/dY1)/2, d/dY = d/dY1 + d/dY2 with the
// five-point weights along each index):
//   res += (D2 - D1)(T5 + T6)/2 + (D1 + D2)(T9 + T10 + T11) - (T12 + T13 + T14),
// T14 = -2 (eps(Y1) + eps(Y2)).  Same block order as k_fd_terms (tiles of
// FD_TY rows Y1 per Y2, chunks of the plane fastest, XCD-contiguous ranges).
__global__ __launch_bounds__(256) void k_resid(OutPtrs out, const double *__restrict__ prof,
                                               Dims d, Tables t, int nchunk)
{
    const int ny = d.ny;
    const size_t plane = (size_t)d.nqo * d.npo;   // output map points per pair
    const int nb = (int)gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7;
    const int item = xcd * q8 + min(xcd, r8) + (int)(blockIdx.x >> 3);
    const int chunk = item % nchunk, r = item / nchunk;
    const int yi = r % FD_TY, j2 = (r / FD_TY) % ny, tile = r / (FD_TY * ny);
    const int j1 = tile * FD_TY + yi;
    const size_t i = (size_t)chunk * blockDim.x + threadIdx.x;
    if (j1 >= ny || i >= plane) return;
    const int f = out.f32;
    const int a1 = t.j0[j1], a2 = t.j0[j2];
    // flux maps of one point: Phi_ry = T5 + T6, phi = T9 + T10 + T11
    auto phi_ry = [&](size_t q) { return get(out.t[4], q, f) + get(out.t[5], q, f); };
    auto phi_y = [&](size_t q) {
        return get(out.t[8], q, f) + get(out.t[9], q, f) + get(out.t[10], q, f);
    };
    double y1 = 0.0, y2 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const size_t o1 = ((size_t)(a1 + a) * ny + j2) * plane + i;
        const size_t o2 = ((size_t)j1 * ny + a2 + a) * plane + i;
        const double w1 = t.w5[j1 * 5 + a], w2 = t.w5[j2 * 5 + a];
        y1 += w1 * phi_ry(o1);
        y2 += w2 * phi_ry(o2);
        f1 += w1 * phi_y(o1);
        f2 += w2 * phi_y(o2);
    }
    const size_t o = ((size_t)j1 * ny + j2) * plane + i;
    const double *eps = prof + P_EPS * ny;
    const double xi = get(out.t[11], o, f) + get(out.t[12], o, f) - 2.0 * (eps[j1] + eps[j2]);
    put(out.res, o, get(out.res, o, f) + 0.5 * (y2 - y1) + f1 + f2 - xi, f);
}

hipError_t launch_resid(hipStream_t st, const Dims &d, const Tables &t, void *const *out,
                        int f32, const double *prof, void *resid)
{
    const size_t plane = (size_t)d.nqo * d.npo;   // output map points per pair
    const int nchunk = (int)((plane + 255) / 256);
    const size_t nblk = (size_t)nchunk * d.ny * ((d.ny + FD_TY - 1) / FD_TY) * FD_TY;
    if (nblk >= ((size_t)1 << 31)) return hipErrorInvalidValue;
    OutPtrs op;
    for (int k = 0; k < 14; ++k) op.t[k] = out[k];
    op.res = resid;
    op.f32 = f32;
    for (int k : {4, 5, 8, 9, 10, 11, 12})
        if (!op.t[k]) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_resid, dim3((unsigned)nblk), dim3(256), 0, st, op, prof, d, t, nchunk);
    return hipGetLastError();
}

// Output of one slab in the general modes.  The maps of the slab's rows, of
// their five-point neighbours and (with the mirror average) of the reflected
// rows sit in the full-plane buffer mf[slot][row][Y2][rz][rx < Nx] for the
// eleven terms that come from the transforms (slot k of term t: kslot below).
// For every output pair (Y1, Y2) of the slab (opairs[q] = Y1 | Y2 << 16) and
// every kept separation (rz = rzk[row], rx = rxk[c] < the domain's width; all
// of them without the rx/rz undersampling):
//   mirror = 1: the average with the reflected pair,
//     (T(Y1, Y2) + sigma_y T(2h - Y1, 2h - Y2)) / 2   (Section "Step 2": the
//     other half of the channel doubles the sample; sigma_y = sign of the term
//     under the reflection, Section "Exploiting symmetries");
//   T6, T11 from the five-point Y1 and Y2 derivatives of the (averaged) <du^2>
//   (Section "Step 3"), T14 from eps.
// out[t][(q nqo + row) npo + c]; T14 out[13][q].  The derivatives along Y
// are pointwise in r, so the undersampling drops output points only.
struct OutPtrs14 {
    void *t[14];
    int f32;
};

__global__ __launch_bounds__(256) void k_slab_out(const double *__restrict__ mf, size_t mstride,
                                                  Dims d, Tables t,
                                                  const int *__restrict__ opairs,
                                                  const double *__restrict__ prof, int mirror,
                                                  OutPtrs14 out)
{
    // slot of each term in mf (-1: not a transformed map)
    constexpr int kslot[14] = {0, 1, 2, 3, 4, -1, 5, 6, 7, 8, -1, 9, 10, -1};
    constexpr double sig[14] = {1, 1, 1, 1, -1, -1, 1, 1, -1, -1, -1, 1, 1, 1};
    const int ny = d.ny, nz = d.nz, nx = d.nx;
    const int q = blockIdx.x, row = blockIdx.y, rz = t.rzk[row];   // a kept rz row
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
    for (int c = threadIdx.x; c < d.npo; c += blockDim.x) {
        const int rx = t.rxk[c];   // a kept rx column of the domain's width
        const size_t ofs = (size_t)rz * nx + rx;
        const size_t o = ((size_t)q * d.nqo + row) * d.npo + c;
#pragma unroll
        for (int k = 0; k < 14; ++k)
            if (kslot[k] >= 0 && out.t[k]) put(out.t[k], o, Tb(kslot[k], j1, j2, ofs, sig[k]), out.f32);
        if (fd) {
            double d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                d1 += t.w5[j1 * 5 + a] * Tb(0, a1 + a, j2, ofs, 1.0);
                d2 += t.w5[j2 * 5 + a] * Tb(0, j1, a2 + a, ofs, 1.0);
            }
            if (out.t[5]) put(out.t[5], o, -d.nu * (d2 - d1), out.f32);
            if (out.t[10]) put(out.t[10], o, -0.5 * d.nu * (d1 + d2), out.f32);
        }
    }
    if (out.t[13] && row == 0 && threadIdx.x == 0) {
        const double *eps = prof + P_EPS * ny;
        double v = -2.0 * (eps[j1] + eps[j2]);
        if (mirror) v = 0.5 * (v - 2.0 * (eps[ny - 1 - j1] + eps[ny - 1 - j2]));
        put(out.t[13], q, v, out.f32);
    }
}

hipError_t launch_slab_out(hipStream_t st, const Dims &d, const Tables &t, const double *mf,
                           size_t mstride, const int *opairs, int nopairs, const double *prof,
                           int mirror, void *const *out, int f32)
{
    OutPtrs14 op;
    for (int i = 0; i < 14; ++i) op.t[i] = out[i];
    op.f32 = f32;
    if (nopairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slab_out, dim3(nopairs, d.nqo), dim3(256), 0, st, mf, mstride, d, t,
                       opairs, prof, mirror, op);
    return hipGetLastError();
}

}  // namespace gke
