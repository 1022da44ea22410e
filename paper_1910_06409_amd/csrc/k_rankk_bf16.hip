// k_rankk_bf16.hip -- the cross-spectral update of k_rankk.hip with split-BF16
// three-term MFMA products and FP32 accumulation.
//
// Every spectral value x is stored as x ~ hi + lo with hi = RN_bf16(x) and
// lo = RN_bf16(x - hi).  A real product a b is taken as ah bh + ah bl + al bh
// (the al bl term, below 2^-16 |a b|, is dropped).  For the complex product
// conj(L) R of one snapshot the six real terms of each output part form one
// group of eight K entries (two zero):
//   A    = [Lrh, Lrh, Lrl, Lih, Lih, Lil, 0, 0]
//   B_re = [Rrh, Rrl, Rrh, Rih, Ril, Rih, 0, 0]   -> sum = Re conj(L) R
//   B_im = [Rih, Ril, Rih,-Rrh,-Rrl,-Rrh, 0, 0]   -> sum = Im conj(L) R
// v_mfma_f32_16x16x32_bf16 takes K = 32: lane l carries K entries 8(l/16)..+7,
// so lane group g = l/16 carries snapshot s0 + g and one MFMA covers four
// snapshots.  Rows (Y1) and columns (Y2) are planes, l%16 within the tile.
// Output (checked on the device): lane l, register v -> (row 4(l/16) + v, col l%16).
// The 27 products and nine accumulators are those of k_rankk.hip.
#include "rankk_common.h"

namespace gke {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 as_bf8(unsigned int d0, unsigned int d1, unsigned int d2)
{
    return __builtin_bit_cast(bf8, u4{d0, d1, d2, 0u});
}

// the three operand forms of one stored value (re = rh | rl<<16, im = ih | il<<16)
struct OpA {
    bf8 a;
};
struct OpB {
    bf8 re, im;
};

__device__ __forceinline__ OpA make_a(unsigned int re, unsigned int im)
{
    // [rh, rh, rl, ih, ih, il, 0, 0]
    return OpA{as_bf8((re & 0xffffu) | (re << 16), (re >> 16) | (im << 16), im)};
}
__device__ __forceinline__ OpA neg_a(OpA x)
{
    u4 v = __builtin_bit_cast(u4, x.a);
    v.x ^= 0x80008000u;
    v.y ^= 0x80008000u;
    v.z ^= 0x80008000u;
    return OpA{__builtin_bit_cast(bf8, v)};
}
__device__ __forceinline__ OpB make_b(unsigned int re, unsigned int im)
{
    const unsigned int rre = (re >> 16) | (re << 16);  // [rl, rh]
    const unsigned int rim = (im >> 16) | (im << 16);  // [il, ih]
    OpB b;
    // [rh, rl, rh, ih, il, ih, 0, 0]
    b.re = as_bf8(re, (re & 0xffffu) | (im << 16), rim);
    // [ih, il, ih, -rh, -rl, -rh, 0, 0]
    b.im = as_bf8(im, (im & 0xffffu) | ((re ^ 0x8000u) << 16), rre ^ 0x80008000u);
    return b;
}

__device__ __forceinline__ float hi_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float lo_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ unsigned int bf16_rn(float x)
{
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ unsigned int split_f(float x)
{
    const unsigned int h = bf16_rn(x);
    return h | (bf16_rn(x - __uint_as_float(h << 16)) << 16);
}
// q = (Qxx + Qyy + Qzz) / 5 from the stored hi + lo values, split again
__device__ __forceinline__ void make_q(const bf16x4 *F, unsigned int &re, unsigned int &im)
{
    const float qr = 0.2f * ((hi_f(F[F_QXX].re) + lo_f(F[F_QXX].re)) +
                             (hi_f(F[F_QYY].re) + lo_f(F[F_QYY].re)) +
                             (hi_f(F[F_QZZ].re) + lo_f(F[F_QZZ].re)));
    const float qi = 0.2f * ((hi_f(F[F_QXX].im) + lo_f(F[F_QXX].im)) +
                             (hi_f(F[F_QYY].im) + lo_f(F[F_QYY].im)) +
                             (hi_f(F[F_QZZ].im) + lo_f(F[F_QZZ].im)));
    re = split_f(qr);
    im = split_f(qi);
}

#define GKE_MFMA_BF(c, A, B)                                                          \
    do {                                                                              \
        ar[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((A).a, (B).re, ar[c], 0, 0, 0); \
        ai[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((A).a, (B).im, ai[c], 0, 0, 0); \
    } while (0)

// Loads of one snapshot quad (lane group g takes snapshot s0 + g): a
// wave-uniform base (wavenumber, field, quad) plus a 32-bit lane offset.  A
// snapshot past the end reloads the last valid one (zeroed at use).
__device__ __forceinline__ void load_raw(bf16x4 *L, bf16x4 *R, const char *kb, size_t fbytes,
                                         unsigned loff, unsigned roff, unsigned sbytes, int s0,
                                         int g, int nsnap)
{
    const int s = s0 + g < nsnap ? s0 + g : nsnap - 1;
    const unsigned so = (unsigned)(s - s0) * sbytes;
    const char *base = kb + (size_t)s0 * sbytes;
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        const char *bf = base + f * fbytes;
        const unsigned lo = loff + so, ro = roff + so;
        L[f] = *reinterpret_cast<const bf16x4 *>(bf + lo);
        R[f] = *reinterpret_cast<const bf16x4 *>(bf + ro);
    }
}

// The split products of one snapshot quad into the nine accumulators.
__device__ __forceinline__ void rankk_bf16_step(f4 *ar, f4 *ai, bf16x4 *Lc, const bf16x4 *Rc,
                                                bool ok)
{
    // a snapshot past the end contributes nothing: zero its left operand
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        Lc[f].re = ok ? Lc[f].re : 0u;
        Lc[f].im = ok ? Lc[f].im : 0u;
    }
    unsigned int lqr, lqi, rqr, rqi;
    make_q(Lc, lqr, lqi);
    make_q(Rc, rqr, rqi);
    const OpA u_ = make_a(Lc[F_U].re, Lc[F_U].im), v_ = make_a(Lc[F_V].re, Lc[F_V].im);
    const OpA w_ = make_a(Lc[F_W].re, Lc[F_W].im), p_ = make_a(Lc[F_P].re, Lc[F_P].im);
    const OpA q_ = make_a(lqr, lqi);
    const OpA Qxx = make_a(Lc[F_QXX].re, Lc[F_QXX].im), Qyy = make_a(Lc[F_QYY].re, Lc[F_QYY].im);
    const OpA Qzz = make_a(Lc[F_QZZ].re, Lc[F_QZZ].im), Qxy = make_a(Lc[F_QXY].re, Lc[F_QXY].im);
    const OpA Qxz = make_a(Lc[F_QXZ].re, Lc[F_QXZ].im), Qyz = make_a(Lc[F_QYZ].re, Lc[F_QYZ].im);
    const OpA nu_ = neg_a(u_), nv_ = neg_a(v_), nw_ = neg_a(w_);
    const OpB U = make_b(Rc[F_U].re, Rc[F_U].im), V = make_b(Rc[F_V].re, Rc[F_V].im);
    const OpB W = make_b(Rc[F_W].re, Rc[F_W].im), P = make_b(Rc[F_P].re, Rc[F_P].im);
    const OpB Q = make_b(rqr, rqi);
    const OpB RQxx = make_b(Rc[F_QXX].re, Rc[F_QXX].im), RQyy = make_b(Rc[F_QYY].re, Rc[F_QYY].im);
    const OpB RQzz = make_b(Rc[F_QZZ].re, Rc[F_QZZ].im), RQxy = make_b(Rc[F_QXY].re, Rc[F_QXY].im);
    const OpB RQxz = make_b(Rc[F_QXZ].re, Rc[F_QXZ].im), RQyz = make_b(Rc[F_QYZ].re, Rc[F_QYZ].im);

    GKE_MFMA_BF(0, u_, U);
    GKE_MFMA_BF(1, Qxx, U);
    GKE_MFMA_BF(2, Qxz, U);
    GKE_MFMA_BF(3, Qxy, U);
    GKE_MFMA_BF(8, v_, U);
    GKE_MFMA_BF(4, u_, RQxy);
    GKE_MFMA_BF(1, nu_, RQxx);
    GKE_MFMA_BF(2, nu_, RQxz);
    GKE_MFMA_BF(5, v_, Q);
    GKE_MFMA_BF(0, v_, V);
    GKE_MFMA_BF(1, Qxy, V);
    GKE_MFMA_BF(2, Qyz, V);
    GKE_MFMA_BF(3, Qyy, V);
    GKE_MFMA_BF(6, p_, V);
    GKE_MFMA_BF(7, u_, V);
    GKE_MFMA_BF(4, v_, RQyy);
    GKE_MFMA_BF(5, q_, V);
    GKE_MFMA_BF(1, nv_, RQxy);
    GKE_MFMA_BF(2, nv_, RQyz);
    GKE_MFMA_BF(6, v_, P);
    GKE_MFMA_BF(0, w_, W);
    GKE_MFMA_BF(1, Qxz, W);
    GKE_MFMA_BF(2, Qzz, W);
    GKE_MFMA_BF(3, Qyz, W);
    GKE_MFMA_BF(4, w_, RQyz);
    GKE_MFMA_BF(1, nw_, RQxz);
    GKE_MFMA_BF(2, nw_, RQzz);
}

#ifndef GKE_RANKK16_PF
#define GKE_RANKK16_PF 0
#endif
#ifndef GKE_RANKK16_MINW
#define GKE_RANKK16_MINW 3
#endif

__global__ __launch_bounds__(64, GKE_RANKK16_MINW) void k_rankk_bf16x3(
    const bf16x4 *__restrict__ spec, Dims d, const int *__restrict__ tile_a,
    const int *__restrict__ tile_b, const int *__restrict__ t_rowplane, int nsnap,
    int accumulate, int total, cx<double> *__restrict__ acc)
{
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int Lg = (bid & 7) * (G >> 3) + (bid >> 3);   // XCD-aware order
    if (Lg >= total) return;
    const int k = Lg / d.ntp;
    const int tp = Lg - k * d.ntp;
    const int ta = tile_a[tp], tb = tile_b[tp];

    const int lane = threadIdx.x;
    const int row = lane & 15, g = lane >> 4;
    const size_t fstride = (size_t)d.chunk * d.ny;
    const char *kb = reinterpret_cast<const char *>(spec + (size_t)k * NFIELD * fstride);
    const size_t fbytes = fstride * sizeof(bf16x4);
    const unsigned sbytes = (unsigned)d.ny * sizeof(bf16x4);
    const unsigned loff = (unsigned)t_rowplane[ta * 16 + row] * sizeof(bf16x4);
    const unsigned roff = (unsigned)(tb * 16 + row) * sizeof(bf16x4);

    f4 ar[9], ai[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        ar[c] = f4{0.f, 0.f, 0.f, 0.f};
        ai[c] = f4{0.f, 0.f, 0.f, 0.f};
    }

#if GKE_RANKK16_PF
    bf16x4 Lc[NFIELD], Rc[NFIELD];
    load_raw(Lc, Rc, kb, fbytes, loff, roff, sbytes, 0, g, nsnap);
    for (int s0 = 0; s0 < nsnap; s0 += 4) {
        bf16x4 Ln[NFIELD], Rn[NFIELD];
        load_raw(Ln, Rn, kb, fbytes, loff, roff, sbytes, s0 + 4 < nsnap ? s0 + 4 : s0, g, nsnap);
        __builtin_amdgcn_sched_barrier(0);
        rankk_bf16_step(ar, ai, Lc, Rc, s0 + g < nsnap);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            Lc[f] = Ln[f];
            Rc[f] = Rn[f];
        }
    }
#else
    for (int s0 = 0; s0 < nsnap; s0 += 4) {
        bf16x4 Lc[NFIELD], Rc[NFIELD];
        load_raw(Lc, Rc, kb, fbytes, loff, roff, sbytes, s0, g, nsnap);
        rankk_bf16_step(ar, ai, Lc, Rc, s0 + g < nsnap);
    }
#endif

    const size_t sp_stride = (size_t)d.nk * d.npair;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t o = (size_t)k * d.npair + (size_t)tp * 256 + (4 * g + v) * 16 + row;
        double cr[9], ci[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            cr[c] = (double)ar[c][v];
            ci[c] = (double)ai[c][v];
        }
        store_spectra(acc, sp_stride, o, cr, ci, accumulate);
    }
}

hipError_t launch_rankk_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                               const bf16x4 *spec, int nsnap, int accumulate, cx<double> *acc)
{
    if (d.ntp > 0) {
        const long long total = (long long)d.nk * d.ntp;
        if (total >= (1LL << 31) - 8) return hipErrorInvalidValue;
        const int G = (int)((total + 7) / 8 * 8);
        hipLaunchKernelGGL(k_rankk_bf16x3, dim3(G), dim3(64), 0, st, spec, d, t.tile_a, t.tile_b,
                           t.rowplane, nsnap, accumulate, (int)total, acc);
    }
    return hipGetLastError();
}

hipError_t launch_rankk_rem_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                                   const bf16x4 *spec, int nsnap, int accumulate,
                                   cx<double> *acc)
{
    return launch_rankk_rem(st, d, t, spec, nsnap, accumulate, acc);
}

}  // namespace gke
