// k_rankk_bf16.hip -- the cross-spectral update of k_rankk.hip with split-BF16
// MFMA products and FP32 accumulation.
//
// Every spectral value x is stored as x ~ hi + lo with hi = RN_bf16(x) and
// lo = RN_bf16(x - hi); a real product a b is taken as ah bh + ah bl + al bh
// (the al bl term, below 2^-16 |a b|, is dropped).  A stored dword holds one
// (re, im) pair of BF16 values, h = (re_hi, im_hi) or l = (re_lo, im_lo), and
// a 32-byte record holds one plane's h dwords of four consecutive snapshots,
// then their l dwords (SplitRec).  For conj(L) R summed over snapshots, the dot
// product of two h dwords is Re(conj(Lh) Rh) of one snapshot, and with the
// right dword rotated, s(re, im) = (im, -re), it is Im(conj(Lh) Rh).
//
// v_mfma_f32_16x16x32_bf16 takes K = 32: lane l carries K entries 8(l/16)..+7,
// i.e. four dwords.  Lane group g = l/16 takes quad q0 + g, so one MFMA sums
// 16 snapshots with every K entry in use, and its operands are whole loaded
// records: per product and part (Re, Im) three MFMAs, (Lh, Rh), (Lh, Rl),
// (Ll, Rh), per 16 snapshots.  Rows (Y1) and columns (Y2) are planes, l%16
// within the tile.  Output (checked on the device): lane l, register v ->
// (row 4(l/16) + v, col l%16).
// The nine accumulators are those of k_rankk.hip; q never enters as a field:
// c5 = (v, q) + (q, v) = 0.2 sum_i [(v, Q_ii) + (Q_ii, v)], 31 products per
// snapshot, which costs four products more and saves forming q from split
// values.  The products are grouped by their right field, whose rotated forms
// are made once per group of 16 snapshots.
#include "rankk_common.h"

namespace gke {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// swap the BF16 halves, negate the new upper one: (a, b) -> (b, -a)
__device__ __forceinline__ unsigned int swapneg(unsigned int x)
{
    return ((x >> 16) | (x << 16)) ^ 0x80000000u;
}
__device__ __forceinline__ u4 swapneg4(u4 x)
{
    return u4{swapneg(x.x), swapneg(x.y), swapneg(x.z), swapneg(x.w)};
}
__device__ __forceinline__ bf8 as_bf8(u4 x) { return __builtin_bit_cast(bf8, x); }

__device__ __forceinline__ f4 mfma(u4 a, u4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf8(a), as_bf8(b), c, 0, 0, 0);
}

// One right field of 16 snapshots and its rotated forms (for the Im part).
struct RightField {
    u4 h, l, sh, sl;
};
__device__ __forceinline__ RightField right_field(u4 h, u4 l)
{
    return RightField{h, l, swapneg4(h), swapneg4(l)};
}
// conj(L) R into channel c: Re with (h, l), Im with the rotated forms
__device__ __forceinline__ void prod(f4 *ar, f4 *ai, int c, u4 ah, u4 al, const RightField &r)
{
    ar[c] = mfma(ah, r.h, ar[c]);
    ai[c] = mfma(ah, r.sh, ai[c]);
    ar[c] = mfma(ah, r.l, ar[c]);
    ai[c] = mfma(ah, r.sl, ai[c]);
    ar[c] = mfma(al, r.h, ar[c]);
    ai[c] = mfma(al, r.sh, ai[c]);
}

// The products of right field B over one group of 16 snapshots (31 in all
// over the ten right fields); the products that enter c1 and c2 with a minus
// sign go to accumulators 9 and 10 of their own, subtracted in the FP64
// epilogue (no negated copies of the left records).
template <int B>
__device__ __forceinline__ void group_products(f4 *ar, f4 *ai, const u4 *LH, const u4 *LL, u4 rh,
                                               u4 rl)
{
    const RightField r = right_field(rh, rl);
    if constexpr (B == F_U) {
        prod(ar, ai, 0, LH[F_U], LL[F_U], r);
        prod(ar, ai, 1, LH[F_QXX], LL[F_QXX], r);
        prod(ar, ai, 2, LH[F_QXZ], LL[F_QXZ], r);
        prod(ar, ai, 3, LH[F_QXY], LL[F_QXY], r);
        prod(ar, ai, 8, LH[F_V], LL[F_V], r);
    } else if constexpr (B == F_V) {
        prod(ar, ai, 0, LH[F_V], LL[F_V], r);
        prod(ar, ai, 1, LH[F_QXY], LL[F_QXY], r);
        prod(ar, ai, 2, LH[F_QYZ], LL[F_QYZ], r);
        prod(ar, ai, 3, LH[F_QYY], LL[F_QYY], r);
        prod(ar, ai, 5, LH[F_QXX], LL[F_QXX], r);
        prod(ar, ai, 5, LH[F_QYY], LL[F_QYY], r);
        prod(ar, ai, 5, LH[F_QZZ], LL[F_QZZ], r);
        prod(ar, ai, 6, LH[F_P], LL[F_P], r);
        prod(ar, ai, 7, LH[F_U], LL[F_U], r);
    } else if constexpr (B == F_W) {
        prod(ar, ai, 0, LH[F_W], LL[F_W], r);
        prod(ar, ai, 1, LH[F_QXZ], LL[F_QXZ], r);
        prod(ar, ai, 2, LH[F_QZZ], LL[F_QZZ], r);
        prod(ar, ai, 3, LH[F_QYZ], LL[F_QYZ], r);
    } else if constexpr (B == F_P) {
        prod(ar, ai, 6, LH[F_V], LL[F_V], r);
    } else if constexpr (B == F_QXX) {
        prod(ar, ai, 9, LH[F_U], LL[F_U], r);
        prod(ar, ai, 5, LH[F_V], LL[F_V], r);
    } else if constexpr (B == F_QYY) {
        prod(ar, ai, 4, LH[F_V], LL[F_V], r);
        prod(ar, ai, 5, LH[F_V], LL[F_V], r);
    } else if constexpr (B == F_QZZ) {
        prod(ar, ai, 10, LH[F_W], LL[F_W], r);
        prod(ar, ai, 5, LH[F_V], LL[F_V], r);
    } else if constexpr (B == F_QXY) {
        prod(ar, ai, 9, LH[F_V], LL[F_V], r);
        prod(ar, ai, 4, LH[F_U], LL[F_U], r);
    } else if constexpr (B == F_QXZ) {
        prod(ar, ai, 9, LH[F_W], LL[F_W], r);
        prod(ar, ai, 10, LH[F_U], LL[F_U], r);
    } else {   // F_QYZ
        prod(ar, ai, 10, LH[F_V], LL[F_V], r);
        prod(ar, ai, 4, LH[F_W], LL[F_W], r);
    }
}

typedef __attribute__((address_space(3))) void lds_void;

// One tile of one group of 16 snapshots in LDS: [field][h, l][lane], 16 bytes
// each, lane l holding plane l%16 of quad l/16 -- the order in which a wave
// loads it and in which the MFMA operands are read back (lane-linear, free of
// bank conflicts).
constexpr int SB_TILE = NFIELD * 2 * 64;   // u4 entries (20 KB)

// One workgroup of four waves per (wavenumber, group of four tile pairs that
// use at most four tiles).  Per group of 16 snapshots every wave copies one
// tile slot into LDS with direct global-to-LDS loads, and each wave then takes
// the operands of its own pair from the slots: a tile shared by two pairs of
// the group is read from L2 once, and the loads hold no registers.  Group s is
// sblk[12 s ..]: four slots (t: row tile t, planes through the row-plane
// table; t | 1 << 16: column tile t; -1: empty), the tile-pair index of each
// wave (-1: none; such a wave still copies its slot and meets the barriers)
// and each wave's left and right slot (l | r << 4).  The 80 KB of LDS let two
// workgroups share a compute unit, one computing while the other waits for
// its copies.  A quad past the end copies the last one and its left operands
// are zeroed (the records of a partial last quad hold zeros in the missing
// snapshots, written by the z pass).
__global__ __launch_bounds__(256, 2) void k_rankk_bf16x3(
    const SplitRec *__restrict__ spec, Dims d, const int *__restrict__ sblk,
    const int *__restrict__ t_rowplane, int nsnap, int accumulate, int total,
    cx<double> *__restrict__ acc)
{
    __shared__ u4 lds[4 * SB_TILE];
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int Lg = (bid & 7) * (G >> 3) + (bid >> 3);   // XCD-aware order
    if (Lg >= total) return;   // whole workgroups
    const int k = Lg / d.nsb;
    const int *sb = sblk + 12 * (Lg - k * d.nsb);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, g = lane >> 4;
    const int nq = (nsnap + 3) >> 2;
    // records of this wavenumber: ((f nqs + q) nys + plane); the field and
    // quad parts are wave-uniform, the plane and lane-group parts a lane offset
    const char *kb = reinterpret_cast<const char *>(spec_base(spec, d, k));
    const size_t fbytes = (size_t)d.nqs * d.nys * sizeof(SplitRec);
    const unsigned qbytes = (unsigned)d.nys * sizeof(SplitRec);
    // the tile this wave copies (slot wv)
    const int code = sb[wv];
    const bool copies = code >= 0;
    const int tile = code & 0xffff;
    const unsigned poff =
        copies ? (unsigned)(code >> 16 ? tile * 16 + row : t_rowplane[tile * 16 + row]) *
                     (unsigned)sizeof(SplitRec)
               : 0u;
    u4 *dst = lds + wv * SB_TILE;
    // the pair of this wave and the slots of its operands
    const int tp = sb[4 + wv];
    const int ops = sb[8 + wv];
    const u4 *Lt = lds + (ops & 15) * SB_TILE + lane;
    const u4 *Rt = lds + (ops >> 4) * SB_TILE + lane;

    // c0 .. c8, then the minus-sign parts of c1 and c2
    f4 ar[11], ai[11];
#pragma unroll
    for (int c = 0; c < 11; ++c) {
        ar[c] = f4{0.f, 0.f, 0.f, 0.f};
        ai[c] = f4{0.f, 0.f, 0.f, 0.f};
    }

    for (int q0 = 0; q0 < nq; q0 += 4) {
        if (copies) {
            // the 32-bit lane offset is formed before it meets the
            // wave-uniform base, so that the loads take the base from scalar
            // registers
            const unsigned lo = poff + (unsigned)min(q0 + g, nq - 1) * qbytes;
#pragma unroll
            for (int f = 0; f < NFIELD; ++f)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    __builtin_amdgcn_global_load_lds(kb + f * fbytes + (lo + 16u * h),
                                                     (lds_void *)(dst + (2 * f + h) * 64), 16,
                                                     0, 0);
        }
        __syncthreads();   // every wave's copies have landed
        if (tp >= 0) {
            const bool ok = q0 + g < nq;
            u4 LH[NFIELD], LL[NFIELD];
#pragma unroll
            for (int f = 0; f < NFIELD; ++f) {
                LH[f] = Lt[(2 * f) * 64];
                LL[f] = Lt[(2 * f + 1) * 64];
            }
            if (!ok) {
#pragma unroll
                for (int f = 0; f < NFIELD; ++f) {
                    LH[f] = u4{0u, 0u, 0u, 0u};
                    LL[f] = u4{0u, 0u, 0u, 0u};
                }
            }
            // each right field is read one group ahead of its products
            u4 rh = Rt[(2 * F_U) * 64], rl = Rt[(2 * F_U + 1) * 64];
#define GKE_GROUP(CUR, NEXT)                                  \
            {                                                 \
                const u4 nh = Rt[(2 * NEXT) * 64];            \
                const u4 nl = Rt[(2 * NEXT + 1) * 64];        \
                group_products<CUR>(ar, ai, LH, LL, rh, rl);  \
                rh = nh;                                      \
                rl = nl;                                      \
                __builtin_amdgcn_sched_barrier(0);            \
            }
            GKE_GROUP(F_U, F_V)
            GKE_GROUP(F_V, F_W)
            GKE_GROUP(F_W, F_P)
            GKE_GROUP(F_P, F_QXX)
            GKE_GROUP(F_QXX, F_QYY)
            GKE_GROUP(F_QYY, F_QZZ)
            GKE_GROUP(F_QZZ, F_QXY)
            GKE_GROUP(F_QXY, F_QXZ)
            GKE_GROUP(F_QXZ, F_QYZ)
#undef GKE_GROUP
            group_products<F_QYZ>(ar, ai, LH, LL, rh, rl);
        }
        __syncthreads();   // every wave has read its operands: the tiles may be refilled
    }
    if (tp < 0) return;

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
        cr[1] -= (double)ar[9][v];
        ci[1] -= (double)ai[9][v];
        cr[2] -= (double)ar[10][v];
        ci[2] -= (double)ai[10][v];
        cr[5] *= 0.2;   // (v, q) + (q, v) from the 0.2 (Q_xx + Q_yy + Q_zz) products
        ci[5] *= 0.2;
        store_spectra(acc, sp_stride, o, cr, ci, accumulate);
    }
}

// One wave per (wavenumber, tile pair), every wave loading its own operands:
// the form for tile-pair sets whose groups of four would leave waves idle
// (a slab with a single row tile, where no column tile is shared and the
// grouped kernel would copy four tiles for three pairs).  Groups of 16
// snapshots (four quads, one per lane group).  A quad past the end reloads
// the last one and its left operands are zeroed (the records of a partial
// last quad hold zeros in the missing snapshots, written by the z pass).
__global__ __launch_bounds__(64, 2) void k_rankk_bf16x3_pair(
    const SplitRec *__restrict__ spec, Dims d, const int *__restrict__ tile_a,
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
    const int nq = (nsnap + 3) >> 2;
    // records of this wavenumber: ((f nqs + q) nys + plane); the field and
    // quad parts are wave-uniform, the plane and lane-group parts a lane offset
    const char *kb = reinterpret_cast<const char *>(spec_base(spec, d, k));
    const size_t fbytes = (size_t)d.nqs * d.nys * sizeof(SplitRec);
    const unsigned qbytes = (unsigned)d.nys * sizeof(SplitRec);
    const unsigned loff = (unsigned)t_rowplane[ta * 16 + row] * sizeof(SplitRec);
    const unsigned roff = (unsigned)(tb * 16 + row) * sizeof(SplitRec);

    // c0 .. c8, then the minus-sign parts of c1 and c2
    f4 ar[11], ai[11];
#pragma unroll
    for (int c = 0; c < 11; ++c) {
        ar[c] = f4{0.f, 0.f, 0.f, 0.f};
        ai[c] = f4{0.f, 0.f, 0.f, 0.f};
    }

    for (int q0 = 0; q0 < nq; q0 += 4) {
        const bool ok = q0 + g < nq;
        const unsigned so = (unsigned)(ok ? g : nq - 1 - q0) * qbytes;
        const char *base = kb + (size_t)q0 * qbytes;
        // the right fields go through three register pairs, each loaded two
        // groups before its products, so that the left records (all ten
        // fields) and three right fields are live at once
        // the 32-bit lane offset is formed before it meets the wave-uniform
        // base, so that the loads take the base from scalar registers
        const unsigned ro = roff + so, lo = loff + so;
        auto ldr = [&](int f, u4 &h, u4 &l) {
            const u4 *rr = reinterpret_cast<const u4 *>(base + f * fbytes + ro);
            h = rr[0];
            l = rr[1];
        };
        u4 h0, l0, h1, l1, h2, l2;
        ldr(F_U, h0, l0);
        ldr(F_V, h1, l1);
        u4 LH[NFIELD], LL[NFIELD];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            const u4 *lr = reinterpret_cast<const u4 *>(base + f * fbytes + lo);
            LH[f] = lr[0];
            LL[f] = lr[1];
        }
        if (!ok) {
#pragma unroll
            for (int f = 0; f < NFIELD; ++f) {
                LH[f] = u4{0u, 0u, 0u, 0u};
                LL[f] = u4{0u, 0u, 0u, 0u};
            }
        }
#define GKE_GROUP(NEXT, HN, LN, CUR, HC, LC)                 \
        ldr(NEXT, HN, LN);                                   \
        group_products<CUR>(ar, ai, LH, LL, HC, LC);         \
        __builtin_amdgcn_sched_barrier(0)
        GKE_GROUP(F_W, h2, l2, F_U, h0, l0);
        GKE_GROUP(F_P, h0, l0, F_V, h1, l1);
        GKE_GROUP(F_QXX, h1, l1, F_W, h2, l2);
        GKE_GROUP(F_QYY, h2, l2, F_P, h0, l0);
        GKE_GROUP(F_QZZ, h0, l0, F_QXX, h1, l1);
        GKE_GROUP(F_QXY, h1, l1, F_QYY, h2, l2);
        GKE_GROUP(F_QXZ, h2, l2, F_QZZ, h0, l0);
        GKE_GROUP(F_QYZ, h0, l0, F_QXY, h1, l1);
#undef GKE_GROUP
        group_products<F_QXZ>(ar, ai, LH, LL, h2, l2);
        group_products<F_QYZ>(ar, ai, LH, LL, h0, l0);
        __builtin_amdgcn_sched_barrier(0);
    }

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
        cr[1] -= (double)ar[9][v];
        ci[1] -= (double)ai[9][v];
        cr[2] -= (double)ar[10][v];
        ci[2] -= (double)ai[10][v];
        cr[5] *= 0.2;   // (v, q) + (q, v) from the 0.2 (Q_xx + Q_yy + Q_zz) products
        ci[5] *= 0.2;
        store_spectra(acc, sp_stride, o, cr, ci, accumulate);
    }
}

hipError_t launch_rankk_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                               const SplitRec *spec, int nsnap, int accumulate, cx<double> *acc)
{
    if (d.ntp <= 0) return hipSuccess;
    // the grouped kernel unless more than an eighth of its waves would idle
    if (d.nsb > 0 && 8 * (4 * d.nsb - d.ntp) <= d.ntp) {
        const long long total = (long long)d.nk * d.nsb;
        if (total >= (1LL << 31) - 8) return hipErrorInvalidValue;
        const int G = (int)((total + 7) / 8 * 8);
        hipLaunchKernelGGL(k_rankk_bf16x3, dim3(G), dim3(256), 0, st, spec, d, t.sblk,
                           t.rowplane, nsnap, accumulate, (int)total, acc);
    } else {
        const long long total = (long long)d.nk * d.ntp;
        if (total >= (1LL << 31) - 8) return hipErrorInvalidValue;
        const int G = (int)((total + 7) / 8 * 8);
        hipLaunchKernelGGL(k_rankk_bf16x3_pair, dim3(G), dim3(64), 0, st, spec, d, t.tile_a,
                           t.tile_b, t.rowplane, nsnap, accumulate, (int)total, acc);
    }
    return hipGetLastError();
}

hipError_t launch_rankk_rem_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                                   const SplitRec *spec, int nsnap, int accumulate,
                                   cx<double> *acc)
{
    return launch_rankk_rem(st, d, t, spec, nsnap, accumulate, acc);
}

}  // namespace gke
