// k_spectra.hip -- per-snapshot part of the second scan (Section "Step 2"):
// fluctuations about the Step-1 means (FP64), the in-plane products formed in
// physical space (Section "Products instead of correlations"), and the 2-D
// forward transform of every plane, written in the layout the cross-spectral
// update reads.  Also the FP64 one-point moments.  (The pseudo-dissipation is
// formed at finalize from the scale-energy spectra, by the Parseval identity;
// on the split-BF16 path its wall-normal part is summed here instead, from FP64
// five-point differences of the fluctuations: forming it from the split
// spectra, sum_ab w_a w_b <u'(Y_a) u'(Y_b)>, would lose digits to cancellation.)
//
// Normalisation: A^(kx,kz) = (1/(Nx Nz)) sum_{x,z} A e^{-i(alpha x + beta z)}.
#include <algorithm>

#include "gke_internal.h"

namespace gke {

template <typename F>
static void set_lds_limit(F *kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)LDS_BUDGET);
}

// BF16 helpers for the split spectra: round to nearest even (finite inputs)
__device__ __forceinline__ unsigned int bf16_rn_bits(float x)
{
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_bits_to_float(unsigned int h) { return __uint_as_float(h << 16); }
// x ~ hi + lo with hi = RN_bf16(x), lo = RN_bf16(x - hi); packed hi | lo << 16
__device__ __forceinline__ unsigned int split_bf16(float x)
{
    const unsigned int h = bf16_rn_bits(x);
    const unsigned int l = bf16_rn_bits(x - bf16_bits_to_float(h));
    return h | (l << 16);
}

template <typename T>
__device__ __forceinline__ void store_spec(cx<double> *spec, size_t i, cx<T> X) { spec[i] = cx<double>{X.x, X.y}; }
// the split dwords of one value: hi = (re_hi, im_hi), lo = (re_lo, im_lo)
__device__ __forceinline__ void split_value(float re, float im, unsigned int &hi, unsigned int &lo)
{
    const unsigned int r = split_bf16(re), m = split_bf16(im);
    hi = (r & 0xffffu) | (m << 16);
    lo = (r >> 16) | (m & 0xffff0000u);
}

// One block = zb consecutive z rows of plane j.  One pass over the inputs:
// fluctuations (FP64), the ten real fields u v w p Qxx Qyy Qzz Qxy Qxz Qyz
// packed two per complex row into LDS, FP64 one-point partial sums and the
// wall-normal gradient energy; then one batched transform (type T) of the
// 5 zb complex rows along x.
//   inter[j][g][f][kx][row]: x-transformed rows (unnormalised) in groups of zg
//   rows (z = g zg + row); a block writes its zb rows of one group
//   momp[j][k][zblk]: FP64 partial sums of q uv pv qu qv qw and (dy u')^2
template <typename TI, typename T, int BLOCK, int NF, bool GY>
__global__ __launch_bounds__(BLOCK, GKE_FFT_WAVES) void k_fluct_xfft(const TI *__restrict__ u,
                                                          const TI *__restrict__ v,
                                                          const TI *__restrict__ w,
                                                          const TI *__restrict__ p,
                                                          const double *__restrict__ prof,
                                                          Dims d, Tables t,
                                                          cx<T> *__restrict__ inter,
                                                          double *__restrict__ momp)
{
    constexpr int CAP = cap_of<BLOCK>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(lds_raw);
    __shared__ double shm[NMOMP * (BLOCK / 64)];
    // NF > 0: the x length as a constant (its plan compiled in)
    const int nx = NF > 0 ? NF : d.nx, ny = d.ny, nz = d.nz, nkx = nx / 2 + 1, zb = d.zb;
    // blocks in the order (j, zblk), zblk fastest; the blocks of one XCD
    // (workgroup i runs on XCD i mod 8) take a contiguous range of it, so the
    // blocks that share a row group of inter write it through one L2
    const int nblk = (int)gridDim.x, q8 = nblk >> 3, r8 = nblk & 7, xcd = blockIdx.x & 7;
    const int item = xcd * q8 + min(xcd, r8) + (int)(blockIdx.x >> 3);
    const int zblk = item % d.nzb, j = item / d.nzb;
    const int z0 = zblk * zb;
    const int bs = fft_stride(nx);
    const size_t npl = (size_t)nx * nz;
    const size_t off = (size_t)j * npl + (size_t)z0 * nx;
    const double U = prof[P_U * ny + j], V = prof[P_V * ny + j];
    const double W = prof[P_W * ny + j], P = prof[P_P * ny + j];
    const int nel = zb * nx;
    // the wall-normal gradient energy from the five-plane stencil: the split
    // path when the first scan did not sum it (means given by the caller)
    constexpr bool kGy = GY;
    // zb nx and nx stay below CAP / 5 (host check): NI elements per thread
    constexpr int NI = (CAP / 5 + BLOCK - 1) / BLOCK;
    constexpr int NG = kGy ? NI : 1;
    const int js = t.j0[j];
    // every load of this thread is issued before any is consumed: the
    // twiddles, the four inputs and, on the split path, the five-plane stencil
    // (unconditional loads at clamped indices, so that no branch separates
    // them; the extra values are dropped)
    TwiddleCopy<T, BLOCK> twc;
    twc.load(tw_of<T>(t, 0), nx);
    TI in[NI][4];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
        const int e = min((int)threadIdx.x + q * BLOCK, nel - 1);
        in[q][0] = u[off + e];
        in[q][1] = v[off + e];
        in[q][2] = w[off + e];
        in[q][3] = p[off + e];
    }
    cx<T> *tw = lds + 5 * zb * bs;
    twc.store(tw, tw_of<T>(t, 0), nx);   // the twiddle loads were issued first
    TI st[NG][3][5];
    if (kGy) {
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            const int e = min((int)threadIdx.x + q * BLOCK, nel - 1);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const size_t o = (size_t)(js + k) * npl + (size_t)z0 * nx + e;
                st[q][0][k] = u[o];
                st[q][1][k] = v[o];
                st[q][2][k] = w[o];
            }
        }
    }
    // every slot is processed; a slot past the end (clamped to the last
    // element) adds nothing to the sums and rewrites the last element's LDS
    // entries with the same values
    double mq = 0, muv = 0, mpv = 0, mqu = 0, mqv = 0, mqw = 0, mgy = 0;
    Walk2 wr(threadIdx.x, BLOCK, nx);   // (row, x)
#pragma unroll
    for (int q = 0; q < NI; ++q) {
        const bool ok = (int)threadIdx.x + q * BLOCK < nel;
        const double a = (double)in[q][0] - U, b = (double)in[q][1] - V;
        const double c = (double)in[q][2] - W, dd = (double)in[q][3] - P;
        const double qq = a * a + b * b + c * c;
        mq += ok ? qq : 0.0;
        muv += ok ? a * b : 0.0;
        mpv += ok ? dd * b : 0.0;
        mqu += ok ? qq * a : 0.0;
        mqv += ok ? qq * b : 0.0;
        mqw += ok ? qq * c : 0.0;
        if (kGy) {
            double gu = 0, gv = 0, gw = 0;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const double wk = t.w5[j * 5 + k];
                gu += wk * ((double)st[q < NG ? q : 0][0][k] - prof[P_U * ny + js + k]);
                gv += wk * ((double)st[q < NG ? q : 0][1][k] - prof[P_V * ny + js + k]);
                gw += wk * ((double)st[q < NG ? q : 0][2][k] - prof[P_W * ny + js + k]);
            }
            mgy += ok ? gu * gu + gv * gv + gw * gw : 0.0;
        }
        // (u,v) (w,p) (Qxx,Qyy) (Qzz,Qxy) (Qxz,Qyz), two real rows per complex row
        const int row = ok ? wr.hi : zb - 1, x = fft_pad(ok ? wr.lo : nx - 1);
        wr.next();
        lds[(0 * zb + row) * bs + x] = cx<T>{(T)a, (T)b};
        lds[(1 * zb + row) * bs + x] = cx<T>{(T)c, (T)dd};
        lds[(2 * zb + row) * bs + x] = cx<T>{(T)(2.0 * a * a + qq), (T)(2.0 * b * b + qq)};
        lds[(3 * zb + row) * bs + x] = cx<T>{(T)(2.0 * c * c + qq), (T)(2.0 * a * b)};
        lds[(4 * zb + row) * bs + x] = cx<T>{(T)(2.0 * a * c), (T)(2.0 * b * c)};
    }
    // the seven partial sums: wave reductions now, the fixed-order sum over
    // the waves and the update of momp after the transform, so that no global
    // round trip sits before the barrier
    static_assert(NMOMP <= 8, "wave_sum8 reduces eight values");
    const double parts[8] = {mq, muv, mpv, mqu, mqv, mqw, mgy, 0.0};
    const double ws = wave_sum8(parts);
    {
        const int lane = threadIdx.x & 63, g = lane >> 3;
        if ((lane & 7) == 0 && g < NMOMP) shm[g * (BLOCK / 64) + (threadIdx.x >> 6)] = ws;
    }
    __syncthreads();
    lds_fft<T, NF, CAP, BLOCK, -1>(lds, 5 * zb, bs, t.px, tw);
    // split the two real transforms: Fa = (Z(k) + conj Z(-k))/2, Fb = (Z(k) - conj Z(-k))/(2i)
    // row group g of zg rows holds this block's rows at r0 .. r0 + zb - 1
    const int zg = d.zg, g = z0 / zg, r0 = z0 - g * zg;
    cx<T> *dst = inter + ((size_t)j * d.nzg + g) * NFIELD * nkx * zg + r0;
    // e = (pr nkx + k) zb + row; zb divides the block size, so row is fixed
    const int lzb = __builtin_ctz(zb), row = threadIdx.x & (zb - 1);
    Walk2 wk(threadIdx.x >> lzb, BLOCK >> lzb, nkx);   // (pr, k)
    for (int e = threadIdx.x; e < 5 * nkx * zb; e += BLOCK) {
        const int pr = wk.hi, k = wk.lo;
        wk.next();
        const cx<T> *R = lds + (pr * zb + row) * bs;
        const cx<T> Z = R[fft_pad(k)];
        const cx<T> Zc = cconj(R[fft_pad(k == 0 ? 0 : nx - k)]);
        const cx<T> Fa = cx<T>{T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
        const cx<T> Fb = cx<T>{T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
        dst[((2 * pr) * nkx + k) * zg + row] = Fa;
        dst[((2 * pr + 1) * nkx + k) * zg + row] = Fb;
    }
    if ((int)threadIdx.x < NMOMP) {   // shm was written before the first barrier
        double r = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) r += shm[threadIdx.x * (BLOCK / 64) + i];
        momp[((size_t)j * NMOMP + threadIdx.x) * d.nzb + zblk] += r;
    }
}

template <typename TI, typename T, bool GY>
static void launch_fx(hipStream_t st, const Dims &d, const Tables &t, const void *u,
                      const void *v, const void *w, const void *p, const double *prof,
                      void *inter, double *momp)
{
    const size_t lds = sizeof(cx<T>) * (5 * (size_t)d.zb * fft_stride(d.nx) + d.nx);
    with_fft_len(d.nx, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        set_lds_limit(k_fluct_xfft<TI, T, FFT_BLOCK, NF, GY>);
        hipLaunchKernelGGL((k_fluct_xfft<TI, T, FFT_BLOCK, NF, GY>), dim3(d.nzb * d.ny),
                           dim3(FFT_BLOCK), lds, st, (const TI *)u, (const TI *)v, (const TI *)w,
                           (const TI *)p, prof, d, t, (cx<T> *)inter, momp);
    });
}

hipError_t launch_fluct_xfft(hipStream_t st, const Dims &d, const Tables &t, int f32, int gy,
                             const void *u, const void *v, const void *w, const void *p,
                             const double *prof, void *inter, double *momp)
{
    const bool sp = d.prec == PREC_BF16X3;
    if (gy && !sp) return hipErrorInvalidValue;   // the FP64 path takes it from the spectra
    if (f32 && sp) {
        if (gy) launch_fx<float, float, true>(st, d, t, u, v, w, p, prof, inter, momp);
        else launch_fx<float, float, false>(st, d, t, u, v, w, p, prof, inter, momp);
    } else if (f32) {
        launch_fx<float, double, false>(st, d, t, u, v, w, p, prof, inter, momp);
    } else if (sp) {
        if (gy) launch_fx<double, float, true>(st, d, t, u, v, w, p, prof, inter, momp);
        else launch_fx<double, float, false>(st, d, t, u, v, w, p, prof, inter, momp);
    } else {
        launch_fx<double, double, false>(st, d, t, u, v, w, p, prof, inter, momp);
    }
    return hipGetLastError();
}

// One block = jb consecutive planes of one field at one kx (two blocks share
// a compute unit): transform along z (type T), scale, and store
// spec[k = kx*Nz + kz][f][slot][j] (planes contiguous) as FP64 complex or split
// BF16.  Work items in the order
// (f, kx, jblk), jblk fastest; the workgroups of one XCD (workgroup i runs on
// XCD i mod 8) take a contiguous range of items, so the items of neighbouring
// kx, which read the two halves of the same cache lines of inter, meet in one
// L2 a few items apart.
template <typename T, typename S, int BLOCK, int NF>
__global__ __launch_bounds__(BLOCK, GKE_FFT_WAVES) void k_zfft_pack_blk(const cx<T> *__restrict__ inter, Dims d,
                                                         Tables t, int slot,
                                                         S *__restrict__ spec)
{
    constexpr int CAP = cap_of<BLOCK>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<T> *lds = reinterpret_cast<cx<T> *>(lds_raw);
    // NF > 0: the z length as a constant (its plan compiled in)
    const int nx = d.nx, ny = d.ny, nz = NF > 0 ? NF : d.nz, nkx = d.nkx, jb = d.jb;
    const int nitem = (int)gridDim.x, q8 = nitem >> 3, r8 = nitem & 7, xcd = blockIdx.x & 7;
    const int item = xcd * q8 + min(xcd, r8) + (int)(blockIdx.x >> 3);
    const int jblk = item % d.njb, kx = (item / d.njb) % nkx, f = item / (d.njb * nkx);
    const int j0 = jblk * jb;
    const int nb = min(jb, ny - j0);
    const int bs = fft_stride(nz);
    const int zg = d.zg, lzg = __builtin_ctz(zg), zm = zg - 1;
    cx<T> *tw = lds + jb * bs;
    // inter[((((j0 + b) nzg + g) NFIELD + f) nkx + kx) zg + row], z = g zg + row
    // offsets within a block stay below 2^31 (jb planes of inter)
    const int szg = NFIELD * nkx * zg, sb = d.nzg * szg;
    const cx<T> *ib = inter + (size_t)j0 * sb + ((size_t)f * nkx + kx) * zg;
    const int cnt = nb * nz;
    {
        // nb * nz <= CAP: every load of this thread is in flight at once.
        // Loads and LDS stores are unconditional, so that no branch holds a
        // load and its wait: a slot past the end takes the last plane's first
        // element and stores it where that element goes (the same value as
        // its own thread stores).  Element e = b nz + z walked without divisions.
        constexpr int MAXE = (CAP + BLOCK - 1) / BLOCK;
        cx<T> x[MAXE];
        Walk2 w(threadIdx.x, BLOCK, nz);   // (b, z)
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nb;
            const int b = ok ? w.hi : nb - 1, z = ok ? w.lo : 0;
            x[q] = ib[b * sb + (z >> lzg) * szg + (z & zm)];
            w.next();
        }
        TwiddleCopy<T, BLOCK> twc;   // in flight with the gathers
        twc.load(tw_of<T>(t, 1), nz);
        twc.store(tw, tw_of<T>(t, 1), nz);
        w = Walk2(threadIdx.x, BLOCK, nz);
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const bool ok = w.hi < nb;
            lds[(ok ? w.hi : nb - 1) * bs + fft_pad(ok ? w.lo : 0)] = x[q];
            w.next();
        }
    }
    __syncthreads();
    lds_fft<T, NF, CAP, BLOCK, -1>(lds, nb, bs, t.pz, tw);
    const double scale = 1.0 / ((double)nx * (double)nz);
    // spec[(((kx nz + kz) NFIELD + f) chunk + slot) ny + j0 + b]; nz * skz < 2^31
    const int skz = NFIELD * d.chunk * d.nys;
    S *sp = spec + (size_t)kx * nz * skz + ((size_t)f * d.chunk + slot) * d.nys + j0;
    Walk2 ws(threadIdx.x, BLOCK, nb);   // (kz, b)
    for (int e = threadIdx.x; e < cnt; e += BLOCK) {
        const cx<T> Y = lds[ws.lo * bs + fft_pad(ws.hi)];
        const cx<double> X = cx<double>{(double)Y.x * scale, (double)Y.y * scale};
        store_spec<double>(sp, ws.hi * skz + ws.lo, X);
        ws.next();
    }
}

template <typename T, typename S, int BLOCK>
static void launch_zp(hipStream_t st, const Dims &d, const Tables &t, const void *inter, int slot,
                      void *spec)
{
    const int nitems = d.njb * d.nkx * NFIELD;
    const size_t lds = sizeof(cx<T>) * ((size_t)d.jb * fft_stride(d.nz) + d.nz);
    with_fft_len(d.nz, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        set_lds_limit(k_zfft_pack_blk<T, S, BLOCK, NF>);
        hipLaunchKernelGGL((k_zfft_pack_blk<T, S, BLOCK, NF>), dim3(nitems), dim3(BLOCK), lds, st,
                           (const cx<T> *)inter, d, t, slot, (S *)spec);
    });
}

hipError_t launch_zfft_pack(hipStream_t st, const Dims &d, const Tables &t, const void *inter,
                            int slot, void *spec)
{
    // (a persistent form with a register prefetch of the next item measured
    // slower on both paths)
    if (d.prec == PREC_BF16X3) return hipErrorInvalidValue;   // records: launch_zfft_rec
    if (d.zpblk == SMALL_BLOCK) launch_zp<double, cx<double>, SMALL_BLOCK>(st, d, t, inter, slot, spec);
    else launch_zp<double, cx<double>, FFT_BLOCK>(st, d, t, inter, slot, spec);
    return hipGetLastError();
}

// Split path: one block = jb planes of one field at one kx for the ng <= 4
// snapshots of quad q, whose x-transformed rows sit in ng buffers of
// `istride` elements: the z transforms of all of them in one batch (FP32),
// then one 32-byte record per (kz, plane), the missing snapshots of a partial
// quad as zeros.  Work items in the order of k_zfft_pack_blk.
template <int BLOCK, int NF>
__global__ __launch_bounds__(BLOCK, GKE_FFT_WAVES) void k_zfft_rec(const cx<float> *__restrict__ inter,
                                                    size_t istride, Dims d, Tables t, int q,
                                                    int ng, SplitRec *__restrict__ spec)
{
    constexpr int CAP = cap_of<BLOCK>();
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<float> *lds = reinterpret_cast<cx<float> *>(lds_raw);
    const int nx = d.nx, ny = d.ny, nz = NF > 0 ? NF : d.nz, nkx = d.nkx, jb = d.jb;
    const int nitem = (int)gridDim.x, q8 = nitem >> 3, r8 = nitem & 7, xcd = blockIdx.x & 7;
    const int item = xcd * q8 + min(xcd, r8) + (int)(blockIdx.x >> 3);
    const int jblk = item % d.njb, kx = (item / d.njb) % nkx, f = item / (d.njb * nkx);
    const int j0 = jblk * jb;
    const int nb = min(jb, ny - j0);
    const int ngb = ng * nb;               // transforms of this block
    const int bs = fft_stride(nz);
    const int zg = d.zg, lzg = __builtin_ctz(zg), zm = zg - 1;
    cx<float> *tw = lds + 4 * jb * bs;
    const int szg = NFIELD * nkx * zg, sb = d.nzg * szg;
    const cx<float> *ib = inter + (size_t)j0 * sb + ((size_t)f * nkx + kx) * zg;
    {
        // ngb * nz <= CAP: every load of this thread is in flight at once;
        // unconditional loads and stores at clamped indices, as in
        // k_zfft_pack_blk.  Element e = (g nb + b) nz + z.
        constexpr int MAXE = (CAP + BLOCK - 1) / BLOCK;
        cx<float> x[MAXE];
        Walk2 w(threadIdx.x, BLOCK, nz);   // (g nb + b, z)
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            const bool ok = w.hi < ngb;
            const int gb = ok ? w.hi : ngb - 1, z = ok ? w.lo : 0;
            const int g = gb / nb, b = gb - g * nb;
            x[i] = ib[g * istride + (size_t)b * sb + (z >> lzg) * szg + (z & zm)];
            w.next();
        }
        TwiddleCopy<float, BLOCK> twc;   // in flight with the gathers
        twc.load(tw_of<float>(t, 1), nz);
        twc.store(tw, tw_of<float>(t, 1), nz);
        w = Walk2(threadIdx.x, BLOCK, nz);
#pragma unroll
        for (int i = 0; i < MAXE; ++i) {
            const bool ok = w.hi < ngb;
            lds[(ok ? w.hi : ngb - 1) * bs + fft_pad(ok ? w.lo : 0)] = x[i];
            w.next();
        }
    }
    __syncthreads();
    lds_fft<float, NF, CAP, BLOCK, -1>(lds, ngb, bs, t.pz, tw);
    const double scale = 1.0 / ((double)nx * (double)nz);
    // record (k = kx nz + kz, f, q, j0 + b): ((k NFIELD + f) nqs + q) nys + j0 + b
    const size_t rkz = (size_t)NFIELD * d.nqs * d.nys;
    SplitRec *sp = spec + (size_t)kx * nz * rkz + ((size_t)f * d.nqs + q) * d.nys + j0;
    Walk2 ws(threadIdx.x, BLOCK, nb);   // (kz, b)
    for (int e = threadIdx.x; e < nz * nb; e += BLOCK) {
        const int kz = ws.hi, b = ws.lo;
        ws.next();
        unsigned int h[4] = {0u, 0u, 0u, 0u}, l[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g < ng) {
                const cx<float> Y = lds[(g * nb + b) * bs + fft_pad(kz)];
                split_value((float)((double)Y.x * scale), (float)((double)Y.y * scale), h[g], l[g]);
            }
        }
        SplitRec *r = sp + (size_t)kz * rkz + b;
        *reinterpret_cast<uint4 *>(r->h) = make_uint4(h[0], h[1], h[2], h[3]);
        *reinterpret_cast<uint4 *>(r->l) = make_uint4(l[0], l[1], l[2], l[3]);
    }
}

hipError_t launch_zfft_rec(hipStream_t st, const Dims &d, const Tables &t, const void *inter,
                           size_t inter_stride, int q, int ng, SplitRec *spec)
{
    if (d.prec != PREC_BF16X3 || ng < 1 || ng > 4 || q < 0 || q >= d.nqs)
        return hipErrorInvalidValue;
    const int nitems = d.njb * d.nkx * NFIELD;
    const size_t lds = sizeof(cx<float>) * (4 * (size_t)d.jb * fft_stride(d.nz) + d.nz);
    with_fft_len(d.nz, [&](auto len) {
        constexpr int NF = decltype(len)::value;
        set_lds_limit(k_zfft_rec<FFT_BLOCK, NF>);
        hipLaunchKernelGGL((k_zfft_rec<FFT_BLOCK, NF>), dim3(nitems), dim3(FFT_BLOCK), lds, st,
                           (const cx<float> *)inter, inter_stride, d, t, q, ng, spec);
    });
    return hipGetLastError();
}

}  // namespace gke
