// k_rankk_bf16.hip -- the cross-spectral update of k_rankk.hip with split-BF16
// three-term MFMA products and FP32 accumulation.
//
// Every spectral value x is stored as x ~ hi + lo with hi = RN_bf16(x) and
// lo = RN_bf16(x - hi); a real product a b is taken as ah bh + ah bl + al bh
// (the al bl term, below 2^-16 |a b|, is dropped).  The stored dwords are
// h = (re_hi, im_hi) and l = (re_lo, im_lo) (bf16x4).  For conj(L) R of one
// snapshot the six real terms of each output part form one group of eight K
// entries (two zero), built from the dwords without arithmetic:
//   A    = [Lh, Lh, Ll, 0]           = [Lrh, Lih, Lrh, Lih, Lrl, Lil, 0, 0]
//   B_re = [Rh, Rl, Rh, 0]           = [Rrh, Rih, Rrl, Ril, Rrh, Rih, 0, 0]
//   B_im = [s(Rh), s(Rl), s(Rh), 0]  = [Rih,-Rrh, Ril,-Rrl, Rih,-Rrh, 0, 0]
// (s(x) swaps the two halves and negates the new upper one):
//   A . B_re = Re conj(L) R,  A . B_im = Im conj(L) R  (three terms each).
// v_mfma_f32_16x16x32_bf16 takes K = 32: lane l carries K entries 8(l/16)..+7,
// so lane group g = l/16 carries snapshot s0 + g and one MFMA covers four
// snapshots.  Rows (Y1) and columns (Y2) are planes, l%16 within the tile.
// Output (checked on the device): lane l, register v -> (row 4(l/16) + v, col l%16).
// The nine accumulators are those of k_rankk.hip; q never enters as a field:
// c5 = (v, q) + (q, v) = 0.2 sum_i [(v, Q_ii) + (Q_ii, v)], 31 products per
// snapshot, which costs four MFMA pairs and saves forming q from split values.
#include "rankk_common.h"

namespace gke {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 op3(unsigned int d0, unsigned int d1, unsigned int d2)
{
    return __builtin_bit_cast(bf8, u4{d0, d1, d2, 0u});
}
// swap the BF16 halves, negate the new upper one: (a, b) -> (b, -a)
__device__ __forceinline__ unsigned int swapneg(unsigned int x)
{
    return ((x >> 16) | (x << 16)) ^ 0x80000000u;
}
constexpr unsigned int NEG2 = 0x80008000u;   // negate both halves

#define GKE_MFMA_BF(c, A, BRE, BIM)                                                \
    do {                                                                           \
        ar[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((A), (BRE), ar[c], 0, 0, 0); \
        ai[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((A), (BIM), ai[c], 0, 0, 0); \
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
__device__ __forceinline__ void rankk_bf16_step(f4 *ar, f4 *ai, const bf16x4 *L,
                                                const bf16x4 *R)
{
    // left operands (planes Y1) and the negated u, v, w
    const bf8 u_ = op3(L[F_U].hi, L[F_U].hi, L[F_U].lo);
    const bf8 v_ = op3(L[F_V].hi, L[F_V].hi, L[F_V].lo);
    const bf8 w_ = op3(L[F_W].hi, L[F_W].hi, L[F_W].lo);
    const bf8 p_ = op3(L[F_P].hi, L[F_P].hi, L[F_P].lo);
    const bf8 xx = op3(L[F_QXX].hi, L[F_QXX].hi, L[F_QXX].lo);
    const bf8 yy = op3(L[F_QYY].hi, L[F_QYY].hi, L[F_QYY].lo);
    const bf8 zz = op3(L[F_QZZ].hi, L[F_QZZ].hi, L[F_QZZ].lo);
    const bf8 xy = op3(L[F_QXY].hi, L[F_QXY].hi, L[F_QXY].lo);
    const bf8 xz = op3(L[F_QXZ].hi, L[F_QXZ].hi, L[F_QXZ].lo);
    const bf8 yz = op3(L[F_QYZ].hi, L[F_QYZ].hi, L[F_QYZ].lo);
    const bf8 nu_ = op3(L[F_U].hi ^ NEG2, L[F_U].hi ^ NEG2, L[F_U].lo ^ NEG2);
    const bf8 nv_ = op3(L[F_V].hi ^ NEG2, L[F_V].hi ^ NEG2, L[F_V].lo ^ NEG2);
    const bf8 nw_ = op3(L[F_W].hi ^ NEG2, L[F_W].hi ^ NEG2, L[F_W].lo ^ NEG2);
    // right operands (planes Y2): real-output and imaginary-output forms
#define GKE_B(f, re, im)                                                     \
    const bf8 re = op3(R[f].hi, R[f].lo, R[f].hi);                           \
    const unsigned int im##h = swapneg(R[f].hi), im##l = swapneg(R[f].lo);   \
    const bf8 im = op3(im##h, im##l, im##h)
    GKE_B(F_U, Ur, Ui);
    GKE_B(F_V, Vr, Vi);
    GKE_B(F_W, Wr, Wi);
    GKE_B(F_P, Pr, Pi);
    GKE_B(F_QXX, XXr, XXi);
    GKE_B(F_QYY, YYr, YYi);
    GKE_B(F_QZZ, ZZr, ZZi);
    GKE_B(F_QXY, XYr, XYi);
    GKE_B(F_QXZ, XZr, XZi);
    GKE_B(F_QYZ, YZr, YZi);
#undef GKE_B
    // 31 products, ordered so that successive ones feed different accumulators
    GKE_MFMA_BF(0, u_, Ur, Ui);
    GKE_MFMA_BF(1, xx, Ur, Ui);
    GKE_MFMA_BF(2, xz, Ur, Ui);
    GKE_MFMA_BF(3, xy, Ur, Ui);
    GKE_MFMA_BF(8, v_, Ur, Ui);
    GKE_MFMA_BF(5, v_, XXr, XXi);
    GKE_MFMA_BF(4, u_, XYr, XYi);
    GKE_MFMA_BF(1, nu_, XXr, XXi);
    GKE_MFMA_BF(2, nu_, XZr, XZi);
    GKE_MFMA_BF(0, v_, Vr, Vi);
    GKE_MFMA_BF(5, xx, Vr, Vi);
    GKE_MFMA_BF(1, xy, Vr, Vi);
    GKE_MFMA_BF(2, yz, Vr, Vi);
    GKE_MFMA_BF(3, yy, Vr, Vi);
    GKE_MFMA_BF(6, p_, Vr, Vi);
    GKE_MFMA_BF(7, u_, Vr, Vi);
    GKE_MFMA_BF(5, yy, Vr, Vi);
    GKE_MFMA_BF(4, v_, YYr, YYi);
    GKE_MFMA_BF(1, nv_, XYr, XYi);
    GKE_MFMA_BF(2, nv_, YZr, YZi);
    GKE_MFMA_BF(6, v_, Pr, Pi);
    GKE_MFMA_BF(5, v_, YYr, YYi);
    GKE_MFMA_BF(0, w_, Wr, Wi);
    GKE_MFMA_BF(1, xz, Wr, Wi);
    GKE_MFMA_BF(2, zz, Wr, Wi);
    GKE_MFMA_BF(3, yz, Wr, Wi);
    GKE_MFMA_BF(5, zz, Vr, Vi);
    GKE_MFMA_BF(4, w_, YZr, YZi);
    GKE_MFMA_BF(1, nw_, XZr, XZi);
    GKE_MFMA_BF(2, nw_, ZZr, ZZi);
    GKE_MFMA_BF(5, v_, ZZr, ZZi);
}

// The products of one snapshot quad; ok = false (a snapshot past the end)
// zeroes the left operand, which folds into the copies that build the MFMA
// operands.
__device__ __forceinline__ void quad_products(f4 *ar, f4 *ai, const bf16x4 *Lq, const bf16x4 *R,
                                              bool ok)
{
    bf16x4 L[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        L[f].hi = ok ? Lq[f].hi : 0u;
        L[f].lo = ok ? Lq[f].lo : 0u;
    }
    rankk_bf16_step(ar, ai, L, R);
}

// Register buffers of snapshot quads: quad q is read from buffer q mod NB,
// which is refilled with quad q + NB right after its last use, so every load
// has NB - 1 quads of products to arrive in.  (A rotating prefetch queue would
// copy the newest buffer down each quad, and a copy waits for its loads.)
#ifndef GKE_RANKK16_NB
#define GKE_RANKK16_NB 3
#endif
#ifndef GKE_RANKK16_MINW
#define GKE_RANKK16_MINW 2
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
    const size_t fstride = (size_t)d.chunk * d.nys;
    const char *kb = reinterpret_cast<const char *>(spec + (size_t)k * NFIELD * fstride);
    const size_t fbytes = fstride * sizeof(bf16x4);
    const unsigned sbytes = (unsigned)d.nys * sizeof(bf16x4);
    const unsigned loff = (unsigned)t_rowplane[ta * 16 + row] * sizeof(bf16x4);
    const unsigned roff = (unsigned)(tb * 16 + row) * sizeof(bf16x4);

    f4 ar[9], ai[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        ar[c] = f4{0.f, 0.f, 0.f, 0.f};
        ai[c] = f4{0.f, 0.f, 0.f, 0.f};
    }

    constexpr int NB = GKE_RANKK16_NB;
    const int nq = (nsnap + 3) >> 2;
    bf16x4 Lb[NB][NFIELD], Rb[NB][NFIELD];
#pragma unroll
    for (int i = 0; i < NB; ++i)
        load_raw(Lb[i], Rb[i], kb, fbytes, loff, roff, sbytes, 4 * min(i, nq - 1), g, nsnap);
    // full groups of NB quads, without branches (a branch around a quad would
    // make the wait before it cover every load in flight)
    int q0 = 0;
    for (; q0 + NB <= nq; q0 += NB) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            quad_products(ar, ai, Lb[i], Rb[i], 4 * (q0 + i) + g < nsnap);
            // the refill is issued after the last read of the buffer
            __builtin_amdgcn_sched_barrier(0);
            load_raw(Lb[i], Rb[i], kb, fbytes, loff, roff, sbytes, 4 * min(q0 + i + NB, nq - 1), g,
                     nsnap);
        }
    }
    // the last nq - q0 < NB quads are in buffers 0, 1, ...
#pragma unroll
    for (int i = 0; i + 1 < NB; ++i)
        if (q0 + i < nq) quad_products(ar, ai, Lb[i], Rb[i], 4 * (q0 + i) + g < nsnap);

    const size_t sp_stride = (size_t)d.nk * d.pstr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t o = (size_t)k * d.pstr + (size_t)tp * 256 + (4 * g + v) * 16 + row;
        double cr[9], ci[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            cr[c] = (double)ar[c][v];
            ci[c] = (double)ai[c][v];
        }
        cr[5] *= 0.2;   // (v, q) + (q, v) from the 0.2 (Q_xx + Q_yy + Q_zz) products
        ci[5] *= 0.2;
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
